// Fused FP32 correlation path: three streaming passes over each rotation's
// grid plus a small per-rotation finish.
//
//  K0 prep          (once per call): max |c_k| -> fixed-point scale.
//  K1 spread_slab   (rotation, z-slab): zero an N x N slab in LDS, scatter
//                   the body samples whose reflected position -R x_k lies
//                   within the B-spline support of this slab, forward 2D
//                   FFT over (x, y) in LDS, one coalesced write of the slab.
//                   The scatter accumulates 32-bit fixed-point values with
//                   LDS integer atomics: on gfx950 these run several times
//                   faster than LDS float atomics, and integer sums do not
//                   depend on the order of the additions, so the spread is
//                   bitwise deterministic.  The scale leaves 8x headroom over
//                   max |c_k| (the B-spline weights of a unit-density lattice
//                   sum to about one at every node); two's-complement
//                   wrap-around of partial sums cancels as long as the final
//                   node value is in range.
//  K2 pencil        (rotation group, pencil pair): forward z-FFT of the
//                   pencils k = (kx, ky) and -k, product with the fixed
//                   spectrum, Hermitian folding of two rotations A, B into
//                   one complex grid Z = H_A + i H_B (H(k) = (Y(k) + conj(Y(-k)))/2
//                   has inverse transform Re f), inverse z-FFT, write.
//  K3 islab_peak    (rotation pair, z-slab): inverse 2D FFT of the folded
//                   slab; Re is rotation A's score slab, Im rotation B's;
//                   per-slab max / lowest-index argmax of each.
//  K4 finish        (rotation, dz): reduce the slab partials to the peak,
//                   evaluate the 9 scores of slab t_z + dz around it by a
//                   separable direct inverse 2D DFT of the folded slab (FP64
//                   accumulation); K5 assembles the 27 values and refines the
//                   peak per axis in FP64.
//
// Correlation form: f(R, t) = sum_p rho_F(p) M_R(p - t) is a circular
// convolution of rho_F with the reflected spread Mr(u) = M_R(-u), i.e. the
// spread of the samples at -R x_k / h.  So fft(f) = S(k) * fft(Mr)(k) with
// S = N^-3 fft(rho_F), and the unnormalised inverse FFT gives f directly.
#include "common.hpp"
#include "fft.hpp"
#include "launch.hpp"

namespace sdf {

namespace {

using cf = cplx<float>;

constexpr int kSlabBlock = 1024;
constexpr int kPencilBlock = 512;
constexpr int kFinishBlock = 256;

template <int N>
constexpr int pencil_width() {
    return N >= 16 ? 16 : N;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// ------------------------------------------------------------------ K1
// ------------------------------------------------------------------ K0
constexpr int kPrepBlocks = 256;

__global__ __launch_bounds__(256) void cmax_partial_kernel(const cf* __restrict__ c, int64_t K,
                                                           float* __restrict__ part) {
    float m = 0.f;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < K; i += int64_t(gridDim.x) * 256) {
        const cf v = c[i];
        m = fmaxf(m, fmaxf(fabsf(v.re), fabsf(v.im)));
    }
    for (int off = warpSize / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    __shared__ float wm[4];
    if (threadIdx.x % warpSize == 0) wm[threadIdx.x / warpSize] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
}

// scale[0] = fixed-point units per unit value, scale[1] = its inverse
__global__ void cmax_final_kernel(const float* __restrict__ part, int n, float* __restrict__ scale) {
    float m = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, part[i]);
    for (int off = warpSize / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (threadIdx.x == 0) {
        // |node sum| <= 8 max|c|  ->  8 max|c| * S <= 2^31
        const float sc = m > 0.f ? 268435456.f / m : 1.f;
        scale[0] = sc;
        scale[1] = 1.f / sc;
    }
}

// ------------------------------------------------------------------ K1
template <int N>
__global__ __launch_bounds__(kSlabBlock) void spread_slab_kernel(const float* __restrict__ Rm,
                                                                 const cf* __restrict__ c, int n_m, int planar,
                                                                 const float* __restrict__ scale,
                                                                 cf* __restrict__ slabs) {
    __shared__ cf slab[N * N];
    __shared__ cf tw[N];
    const int z = blockIdx.x;
    const int rot = blockIdx.y;
    const int nz = planar ? 1 : N;
    fill_twiddles<float, N>(tw);
    int* acc = reinterpret_cast<int*>(slab);  // fixed-point (re, im) pairs
    for (int i = threadIdx.x; i < 2 * N * N; i += kSlabBlock) acc[i] = 0;
    const float S = scale[0];
    __syncthreads();

    // reflected rotation: positions y_k = Rp (k - n_m / 2), Rp = -R
    float Rp[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) Rp[a] = -Rm[9 * rot + a];
    const float half = 0.5f * float(n_m);
    if (planar) {
        const int K = n_m * n_m;
        for (int k = threadIdx.x; k < K; k += kSlabBlock) {
            const cf ck = c[k];
            const float cre = ck.re * S, cim = ck.im * S;
            const float bx = float(k % n_m) - half, by = float(k / n_m) - half;
            const float yx = Rp[0] * bx + Rp[1] * by;
            const float yy = Rp[3] * bx + Rp[4] * by;
            const float fx = floorf(yx), fy = floorf(yy);
            float wx[4], wy[4];
            bspline3_weights(yx - fx, wx);
            bspline3_weights(yy - fy, wy);
            const int ix = int(fx) - 1, iy = int(fy) - 1;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int row = wrap(iy + b, N) * N;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const float wt = wx[a] * wy[b];
                    const int idx = 2 * (row + wrap(ix + a, N));
                    atomicAdd(acc + idx, __float2int_rn(cre * wt));
                    atomicAdd(acc + idx + 1, __float2int_rn(cim * wt));
                }
            }
        }
    } else {
        // dominant body axis of the z row: walk it, enumerate the other two
        int ax = 0;
        float best = fabsf(Rp[6]);
        if (fabsf(Rp[7]) > best) { ax = 1; best = fabsf(Rp[7]); }
        if (fabsf(Rp[8]) > best) { ax = 2; }
        const int b1 = ax == 0 ? 1 : 0;
        const int b2 = ax == 2 ? 1 : 2;
        const float sa = Rp[6 + ax];
        const float zc = float(z < N / 2 ? z : z - N);  // centred image of this slab
        const int pairs = n_m * n_m;
        for (int pidx = threadIdx.x; pidx < pairs; pidx += kSlabBlock) {
            int kk[3];
            kk[b1] = pidx % n_m;
            kk[b2] = pidx / n_m;
            const float base = Rp[6 + b1] * (float(kk[b1]) - half) + Rp[6 + b2] * (float(kk[b2]) - half);
            float lo_f = (zc - 2.f - base) / sa, hi_f = (zc + 2.f - base) / sa;
            if (lo_f > hi_f) { float t = lo_f; lo_f = hi_f; hi_f = t; }
            int lo = int(floorf(lo_f + half)), hi = int(ceilf(hi_f + half));
            lo = lo < 0 ? 0 : lo;
            hi = hi > n_m - 1 ? n_m - 1 : hi;
            for (int ka = lo; ka <= hi; ++ka) {
                kk[ax] = ka;
                const float bx = float(kk[0]) - half, by = float(kk[1]) - half, bz = float(kk[2]) - half;
                const float yz = Rp[6] * bx + Rp[7] * by + Rp[8] * bz;
                const float dz = zc - yz;
                if (!(fabsf(dz) < 2.f)) continue;
                const float yx = Rp[0] * bx + Rp[1] * by + Rp[2] * bz;
                const float yy = Rp[3] * bx + Rp[4] * by + Rp[5] * bz;
                const float ad = fabsf(dz);
                float wz;
                if (ad < 1.f) wz = 2.f / 3.f - ad * ad + 0.5f * ad * ad * ad;
                else { const float b = 2.f - ad; wz = b * b * b / 6.f; }
                const int k = (kk[2] * n_m + kk[1]) * n_m + kk[0];
                const cf ck = c[k];
                const float cre = ck.re * (wz * S), cim = ck.im * (wz * S);
                const float fx = floorf(yx), fy = floorf(yy);
                float wx[4], wy[4];
                bspline3_weights(yx - fx, wx);
                bspline3_weights(yy - fy, wy);
                const int ix = int(fx) - 1, iy = int(fy) - 1;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int row = wrap(iy + b, N) * N;
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const float wt = wx[a] * wy[b];
                        const int idx = 2 * (row + wrap(ix + a, N));
                        atomicAdd(acc + idx, __float2int_rn(cre * wt));
                        atomicAdd(acc + idx + 1, __float2int_rn(cim * wt));
                    }
                }
            }
        }
    }
    __syncthreads();
    const float inv = scale[1];
    for (int i = threadIdx.x; i < N * N; i += kSlabBlock) {
        const int2 v = reinterpret_cast<const int2*>(acc)[i];
        slab[i] = mk(float(v.x) * inv, float(v.y) * inv);
    }
    __syncthreads();
    lds_fft_lines<float, N, -1, false>(slab, 1, N, N, tw);  // along x
    lds_fft_lines<float, N, -1, true>(slab, N, 1, N, tw);   // along y
    cf* out = slabs + (int64_t(rot) * nz + z) * N * N;
    for (int i = threadIdx.x; i < N * N; i += kSlabBlock) out[i] = slab[i];
}

// ------------------------------------------------------------------ K2
struct PencilJob {
    int ky, x0;
};

template <int N>
__device__ __forceinline__ PencilJob pencil_job(int j) {
    constexpr int W = pencil_width<N>();
    constexpr int CH = N / W;
    constexpr int SC = (N / 2 + 1 + W - 1) / W;
    constexpr int full = (N / 2 - 1) * CH;
    if (j < full) return PencilJob{1 + j / CH, (j % CH) * W};
    j -= full;
    return PencilJob{(j / SC) ? N / 2 : 0, (j % SC) * W};
}

template <int N>
constexpr int pencil_jobs() {
    constexpr int W = pencil_width<N>();
    return (N / 2 - 1) * (N / W) + 2 * ((N / 2 + 1 + W - 1) / W);
}

// NZ = N (3D) or 1 (planar); GR rotations per block (2 or 4)
template <int N, int NZ, int GR>
__global__ __launch_bounds__(kPencilBlock) void pencil_kernel(const cf* __restrict__ slabs,
                                                              const cf* __restrict__ spec, int nb,
                                                              cf* __restrict__ packed) {
    constexpr int W = pencil_width<N>();
    constexpr int NL = 2 * W * GR;  // lines: (rotation, tile, column)
    __shared__ cf buf[NZ * NL];
    __shared__ cf tw[NZ > 1 ? NZ : 1];
    const PencilJob job = pencil_job<N>(blockIdx.x);
    const int g0 = blockIdx.y * GR;  // first rotation of the group in the batch
    const int64_t G = int64_t(N) * N * NZ;
    const int kyt[2] = {job.ky, (N - job.ky) % N};
    if constexpr (NZ > 1) fill_twiddles<float, NZ>(tw);

    auto line_of = [](int r, int t, int cc) { return ((r & 1) * GR + (r >> 1) * 2 + t) * W + cc; };
    auto kx_of = [&](int t, int cc) { return t == 0 ? job.x0 + cc : (N - job.x0 - cc) % N; };

    // load both tiles of every rotation of the group (zeros for missing rotations)
    for (int i = threadIdx.x; i < GR * 2 * NZ * W; i += kPencilBlock) {
        const int cc = i % W;
        const int kz = (i / W) % NZ;
        const int t = (i / (W * NZ)) % 2;
        const int r = i / (W * NZ * 2);
        const int rot = g0 + r;
        cf v = mk(0.f, 0.f);
        if (rot < nb) v = slabs[int64_t(rot) * G + (int64_t(kz) * N + kyt[t]) * N + kx_of(t, cc)];
        buf[kz * NL + line_of(r, t, cc)] = v;
    }
    __syncthreads();
    if constexpr (NZ > 1) lds_fft_lines<float, NZ, -1, true>(buf, NL, 1, NL, tw);
    else __syncthreads();
    // product with the fixed spectrum (read once, used by every rotation)
    for (int i = threadIdx.x; i < 2 * NZ * W; i += kPencilBlock) {
        const int cc = i % W;
        const int kz = (i / W) % NZ;
        const int t = i / (W * NZ);
        const cf sv = spec[(int64_t(kz) * N + kyt[t]) * N + kx_of(t, cc)];
#pragma unroll
        for (int r = 0; r < GR; ++r) {
            cf& y = buf[kz * NL + line_of(r, t, cc)];
            y = y * sv;
        }
    }
    __syncthreads();
    // Hermitian folding of rotation pairs: A lines receive Z = H_A + i H_B
    for (int i = threadIdx.x; i < (GR / 2) * NZ * W; i += kPencilBlock) {
        const int cc = i % W;
        const int kz = (i / W) % NZ;
        const int p = i / (W * NZ);
        const int mkz = (NZ - kz) % NZ;
        const int a0 = line_of(2 * p, 0, cc), a1 = line_of(2 * p, 1, cc);
        const int b0 = line_of(2 * p + 1, 0, cc), b1 = line_of(2 * p + 1, 1, cc);
        const cf ya0 = buf[kz * NL + a0], ya1 = buf[mkz * NL + a1];
        const cf yb0 = buf[kz * NL + b0], yb1 = buf[mkz * NL + b1];
        const cf ha = (ya0 + conj(ya1)) * 0.5f;
        const cf hb = (yb0 + conj(yb1)) * 0.5f;
        buf[kz * NL + a0] = mk(ha.re - hb.im, ha.im + hb.re);
        buf[mkz * NL + a1] = mk(ha.re + hb.im, hb.re - ha.im);
    }
    __syncthreads();
    if constexpr (NZ > 1) lds_fft_lines<float, NZ, 1, true>(buf, NL, 1, GR * W, tw);
    // write the folded pencils of each pair
    const int pair0 = g0 / 2;
    const int npair = (nb + 1) / 2;
    for (int i = threadIdx.x; i < (GR / 2) * 2 * NZ * W; i += kPencilBlock) {
        const int cc = i % W;
        const int kz = (i / W) % NZ;
        const int t = (i / (W * NZ)) % 2;
        const int p = i / (W * NZ * 2);
        if (pair0 + p >= npair) continue;
        packed[int64_t(pair0 + p) * G + (int64_t(kz) * N + kyt[t]) * N + kx_of(t, cc)] =
            buf[kz * NL + line_of(2 * p, t, cc)];
    }
}

// ------------------------------------------------------------------ K3
__device__ __forceinline__ bool better(float v, int i, float bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

__device__ __forceinline__ void wave_argmax(float& v, int& i) {
    for (int off = warpSize / 2; off > 0; off >>= 1) {
        const float ov = __shfl_xor(v, off);
        const int oi = __shfl_xor(i, off);
        if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
}

template <int N>
__global__ __launch_bounds__(kSlabBlock) void islab_peak_kernel(const cf* __restrict__ packed, int nz, int nb,
                                                                float* __restrict__ pval, int* __restrict__ pidx) {
    __shared__ cf slab[N * N];
    __shared__ cf tw[N];
    __shared__ float rv[2][kSlabBlock / 64];
    __shared__ int ri[2][kSlabBlock / 64];
    const int z = blockIdx.x, pair = blockIdx.y;
    fill_twiddles<float, N>(tw);
    const cf* src = packed + (int64_t(pair) * nz + z) * N * N;
    for (int i = threadIdx.x; i < N * N; i += kSlabBlock) slab[i] = src[i];
    __syncthreads();
    lds_fft_lines<float, N, 1, true>(slab, N, 1, N, tw);   // along y
    lds_fft_lines<float, N, 1, false>(slab, 1, N, N, tw);  // along x
    float va = -INFINITY, vb = -INFINITY;
    int ia = 0x7fffffff, ib = 0x7fffffff;
    const int zoff = z * N * N;
    for (int i = threadIdx.x; i < N * N; i += kSlabBlock) {
        const cf v = slab[i];
        if (better(v.re, zoff + i, va, ia)) { va = v.re; ia = zoff + i; }
        if (better(v.im, zoff + i, vb, ib)) { vb = v.im; ib = zoff + i; }
    }
    wave_argmax(va, ia);
    wave_argmax(vb, ib);
    const int lane = threadIdx.x % warpSize, wid = threadIdx.x / warpSize;
    if (lane == 0) {
        rv[0][wid] = va;
        ri[0][wid] = ia;
        rv[1][wid] = vb;
        ri[1][wid] = ib;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int w = threadIdx.x;
        float bv = rv[w][0];
        int bi = ri[w][0];
        for (int k = 1; k < kSlabBlock / 64; ++k)
            if (better(rv[w][k], ri[w][k], bv, bi)) { bv = rv[w][k]; bi = ri[w][k]; }
        const int rot = 2 * pair + w;
        if (rot < nb) {
            pval[int64_t(rot) * nz + z] = bv;
            pidx[int64_t(rot) * nz + z] = bi;
        }
    }
}

// ------------------------------------------------------------------ K4
// (dz, rotation): peak from the slab partials, then the 9 scores of slab
// t_z + dz around (t_x, t_y) by a separable inverse DFT of the folded slab:
//   h_j(ky)  = sum_kx P(kx, ky) e^{2 pi i kx x_j / N},  x_j in t_x + {-1, 0, 1}
//   g(x_j, y_i) = sum_ky h_j(ky) e^{2 pi i ky y_i / N}
// Re g belongs to the even rotation of the pair, Im g to the odd one.
template <int N>
__global__ __launch_bounds__(kFinishBlock) void finish_slab_kernel(const cf* __restrict__ packed, int nz,
                                                                   const float* __restrict__ pval,
                                                                   const int* __restrict__ pidx,
                                                                   double* __restrict__ nbbuf,
                                                                   float* __restrict__ score,
                                                                   int32_t* __restrict__ tout) {
    __shared__ float sv[kFinishBlock];
    __shared__ int si[kFinishBlock];
    __shared__ double twr[N], twi[N];
    __shared__ double hre[N][2][3], him[N][2][3];
    __shared__ double red[kFinishBlock / 64][9];
    const int rot = blockIdx.y;
    const int dzi = gridDim.x == 1 ? 1 : blockIdx.x;
    for (int m = threadIdx.x; m < N; m += kFinishBlock) {
        double sn, cs;
        sincospi(2.0 * double(m) / double(N), &sn, &cs);
        twr[m] = cs;
        twi[m] = sn;
    }
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < nz; i += kFinishBlock) {
        const float v = pval[int64_t(rot) * nz + i];
        const int id = pidx[int64_t(rot) * nz + i];
        if (better(v, id, bv, bi)) { bv = v; bi = id; }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kFinishBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off && better(sv[threadIdx.x + off], si[threadIdx.x + off], sv[threadIdx.x], si[threadIdx.x])) {
            sv[threadIdx.x] = sv[threadIdx.x + off];
            si[threadIdx.x] = si[threadIdx.x + off];
        }
        __syncthreads();
    }
    bv = sv[0];
    bi = si[0];
    const int tx = bi % N, ty = (bi / N) % N, tz = bi / (N * N);
    const int zz = wrap(tz + dzi - 1, nz);
    const cf* sl = packed + (int64_t(rot / 2) * nz + zz) * N * N;
    const bool imag = rot & 1;
    const int xs[3] = {(tx + N - 1) % N, tx, (tx + 1) % N};
    const int ys[3] = {(ty + N - 1) % N, ty, (ty + 1) % N};
    // inner sums along x: two threads per row ky, each half of the row
    for (int w = threadIdx.x; w < 2 * N; w += kFinishBlock) {
        const int ky = w >> 1, half = w & 1;
        double ar[3] = {0, 0, 0}, ai[3] = {0, 0, 0};
        for (int kx = half * (N / 2); kx < (half + 1) * (N / 2); ++kx) {
            const cf v = sl[ky * N + kx];
            const double vr = v.re, vi = v.im;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int m = (kx * xs[j]) % N;
                ar[j] += vr * twr[m] - vi * twi[m];
                ai[j] += vr * twi[m] + vi * twr[m];
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            hre[ky][half][j] = ar[j];
            him[ky][half][j] = ai[j];
        }
    }
    __syncthreads();
    double part[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) part[a] = 0.0;
    for (int ky = threadIdx.x; ky < N; ky += kFinishBlock) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double hr = hre[ky][0][j] + hre[ky][1][j];
            const double hi = him[ky][0][j] + him[ky][1][j];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int m = (ky * ys[i]) % N;
                part[i * 3 + j] += imag ? hr * twi[m] + hi * twr[m] : hr * twr[m] - hi * twi[m];
            }
        }
    }
    const int lane = threadIdx.x % warpSize, wid = threadIdx.x / warpSize;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        double v = part[a];
        for (int off = warpSize / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wid][a] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double v = 0.0;
        for (int w = 0; w < kFinishBlock / 64; ++w) v += red[w][threadIdx.x];
        if (gridDim.x == 1) {  // planar: the three z offsets wrap onto the one slab
            for (int d = 0; d < 3; ++d) nbbuf[27 * int64_t(rot) + d * 9 + threadIdx.x] = v;
        } else {
            nbbuf[27 * int64_t(rot) + dzi * 9 + threadIdx.x] = v;
        }
    }
    if (dzi == 1 && threadIdx.x == 0) {
        score[rot] = bv;
        tout[3 * rot] = tx;
        tout[3 * rot + 1] = ty;
        tout[3 * rot + 2] = tz;
    }
}

// per rotation: neighbourhood out, per-axis parabola vertex in FP64
__global__ void finish_rot_kernel(const double* __restrict__ nbbuf, const int32_t* __restrict__ tout, int n_rot,
                                  float* __restrict__ nbhd, double* __restrict__ refined) {
    const int rot = blockIdx.x * blockDim.x + threadIdx.x;
    if (rot >= n_rot) return;
    const double* nb = nbbuf + 27 * int64_t(rot);
    if (nbhd)
        for (int a = 0; a < 27; ++a) nbhd[27 * int64_t(rot) + a] = float(nb[a]);
    if (refined) {
        const double f0 = nb[13];
        const double fm[3] = {nb[12], nb[10], nb[4]};
        const double fp[3] = {nb[14], nb[16], nb[22]};
        for (int a = 0; a < 3; ++a) {
            const double den = fm[a] - 2.0 * f0 + fp[a];
            double d = 0.0;
            if (den < 0.0) {
                d = (fm[a] - fp[a]) / (2.0 * den);
                d = d < -0.5 ? -0.5 : (d > 0.5 ? 0.5 : d);
            }
            refined[3 * rot + a] = double(tout[3 * rot + a]) + d;
        }
    }
}

struct TimerScope {
    KernelTimer* kt;
    hipStream_t s;
    TimerScope(KernelTimer* k, const char* name, hipStream_t st) : kt(k), s(st) {
        if (kt) kt->begin(name, s);
    }
    ~TimerScope() {
        if (kt) kt->end(s);
    }
};

template <int N>
hipError_t fused_impl(const FusedPlan& fp, const float* R, int n_rot, const void* c, const void* spec, void* ws,
                      float* score, int32_t* t, float* nbhd, double* refined, hipStream_t s, KernelTimer* kt) {
    const int nz = fp.planar ? 1 : N;
    const int64_t G = int64_t(N) * N * nz;
    const int npair = (n_rot + 1) / 2;
    char* base = static_cast<char*>(ws);
    cf* slabs = reinterpret_cast<cf*>(base);
    size_t off = align256(sizeof(cf) * G * fp.batch);
    cf* packed = reinterpret_cast<cf*>(base + off);
    off += align256(sizeof(cf) * G * ((fp.batch + 1) / 2));
    float* pval = reinterpret_cast<float*>(base + off);
    off += align256(sizeof(float) * nz * fp.batch);
    int* pidx = reinterpret_cast<int*>(base + off);
    off += align256(sizeof(int) * nz * fp.batch);
    double* nbbuf = reinterpret_cast<double*>(base + off);
    off += align256(sizeof(double) * 27 * fp.batch);
    const float* scale = reinterpret_cast<const float*>(base + off + align256(sizeof(float) * kPrepBlocks));

    const cf* cc = static_cast<const cf*>(c);
    {
        TimerScope ts(kt, "spread_slab", s);
        hipLaunchKernelGGL(spread_slab_kernel<N>, dim3(nz, n_rot), dim3(kSlabBlock), 0, s, R, cc, fp.n_m,
                           fp.planar ? 1 : 0, scale, slabs);
    }
    const int gr = fp.pencil_group;
    const dim3 g2{unsigned(pencil_jobs<N>()), unsigned((n_rot + gr - 1) / gr), 1u};
    const cf* sp = static_cast<const cf*>(spec);
    {
        TimerScope ts(kt, "pencil", s);
        if (fp.planar) {
            if (gr == 4)
                hipLaunchKernelGGL((pencil_kernel<N, 1, 4>), g2, dim3(kPencilBlock), 0, s, slabs, sp, n_rot, packed);
            else
                hipLaunchKernelGGL((pencil_kernel<N, 1, 2>), g2, dim3(kPencilBlock), 0, s, slabs, sp, n_rot, packed);
        } else {
            if (gr == 4)
                hipLaunchKernelGGL((pencil_kernel<N, N, 4>), g2, dim3(kPencilBlock), 0, s, slabs, sp, n_rot, packed);
            else
                hipLaunchKernelGGL((pencil_kernel<N, N, 2>), g2, dim3(kPencilBlock), 0, s, slabs, sp, n_rot, packed);
        }
    }
    {
        TimerScope ts(kt, "islab_peak", s);
        hipLaunchKernelGGL(islab_peak_kernel<N>, dim3(nz, npair), dim3(kSlabBlock), 0, s, packed, nz, n_rot, pval,
                           pidx);
    }
    {
        TimerScope ts(kt, "finish", s);
        const dim3 g4{unsigned(fp.planar ? 1 : 3), unsigned(n_rot), 1u};
        hipLaunchKernelGGL(finish_slab_kernel<N>, g4, dim3(kFinishBlock), 0, s, packed, nz, pval, pidx, nbbuf, score,
                           t);
        hipLaunchKernelGGL(finish_rot_kernel, dim3(unsigned((n_rot + 63) / 64)), dim3(64), 0, s, nbbuf, t, n_rot,
                           nbhd, refined);
    }
    return hipGetLastError();
}

}  // namespace

size_t fused_workspace_bytes(const FusedPlan& fp) {
    const int nz = fp.planar ? 1 : fp.N;
    const int64_t G = int64_t(fp.N) * fp.N * nz;
    return align256(sizeof(cf) * G * fp.batch) + align256(sizeof(cf) * G * ((fp.batch + 1) / 2)) +
           align256(sizeof(float) * nz * fp.batch) + align256(sizeof(int) * nz * fp.batch) +
           align256(sizeof(double) * 27 * fp.batch) + align256(sizeof(float) * kPrepBlocks) + align256(2 * sizeof(float));
}

// Once per call, before the batches: max |c_k| and the fixed-point scale.
hipError_t launch_fused_prep(const FusedPlan& fp, const void* c, void* ws, hipStream_t s) {
    const int nz = fp.planar ? 1 : fp.N;
    const int64_t G = int64_t(fp.N) * fp.N * nz;
    const int64_t K = int64_t(fp.n_m) * fp.n_m * (fp.planar ? 1 : fp.n_m);
    size_t off = align256(sizeof(cf) * G * fp.batch) + align256(sizeof(cf) * G * ((fp.batch + 1) / 2)) +
                 align256(sizeof(float) * nz * fp.batch) + align256(sizeof(int) * nz * fp.batch) +
                 align256(sizeof(double) * 27 * fp.batch);
    float* part = reinterpret_cast<float*>(static_cast<char*>(ws) + off);
    float* scale = reinterpret_cast<float*>(static_cast<char*>(ws) + off + align256(sizeof(float) * kPrepBlocks));
    hipLaunchKernelGGL(cmax_partial_kernel, dim3(kPrepBlocks), dim3(256), 0, s, static_cast<const cf*>(c), K, part);
    hipLaunchKernelGGL(cmax_final_kernel, dim3(1), dim3(256), 0, s, part, kPrepBlocks, scale);
    return hipGetLastError();
}

hipError_t launch_fused_batch(const FusedPlan& fp, const float* R, int n_rot, const void* c, const void* spec,
                              void* ws, float* score, int32_t* t, float* nbhd, double* refined, hipStream_t s,
                              KernelTimer* kt) {
    switch (fp.N) {
        case 8: return fused_impl<8>(fp, R, n_rot, c, spec, ws, score, t, nbhd, refined, s, kt);
        case 16: return fused_impl<16>(fp, R, n_rot, c, spec, ws, score, t, nbhd, refined, s, kt);
        case 32: return fused_impl<32>(fp, R, n_rot, c, spec, ws, score, t, nbhd, refined, s, kt);
        case 64: return fused_impl<64>(fp, R, n_rot, c, spec, ws, score, t, nbhd, refined, s, kt);
        case 96: return fused_impl<96>(fp, R, n_rot, c, spec, ws, score, t, nbhd, refined, s, kt);
        case 128: return fused_impl<128>(fp, R, n_rot, c, spec, ws, score, t, nbhd, refined, s, kt);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sdf
