// Fused FP32 correlation path: three streaming passes over each rotation's
// grid plus a small per-rotation finish.
//
//  K0 prep          (once per call): max |c_k| -> fixed-point scale.
//  K1 spread_slab   (rotation, z-slab): zero an N x N slab in LDS, scatter
//                   the body samples whose reflected position -R x_k lies
//                   within the B-spline support of this slab, forward 2D
//                   FFT over (x, y) in LDS, one coalesced write of the slab.
//                   The scatter accumulates 32-bit fixed-point values with
//                   LDS integer atomics (a node's re and im in one 64-bit
//                   word, one add per node): on gfx950 these run several
//                   times faster than LDS float atomics, and integer sums do
//                   not depend on the order of the additions, so the spread
//                   is bitwise deterministic.  The scale leaves 8x headroom over
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
//                   max / lowest-index argmax of each per wave and slab.
//  K4 finish        (rotation, dz): reduce the wave partials to the peak,
//                   evaluate the 9 scores of slab t_z + dz around it by a
//                   separable direct inverse 2D DFT of the folded slab (FP64
//                   accumulation); K5 assembles the 27 values and refines the
//                   peak per axis in FP64.
//
// Work is described by descriptors: one FusedJob per pair (coefficients,
// spectrum, fixed-point scale, outputs) and one FusedRot per rotation (FP32
// matrix, owning pair, local index), so one launch sequence serves any mix
// of pairs that share the grid size N.  K1-K3 are persistent: a grid sized
// to the device walks the batch's work items with a stride.
//
// Correlation form: f(R, t) = sum_p rho_F(p) M_R(p - t) is a circular
// convolution of rho_F with the reflected spread Mr(u) = M_R(-u), i.e. the
// spread of the samples at -R x_k / h.  So fft(f) = S(k) * fft(Mr)(k) with
// S = N^-3 fft(rho_F), and the unnormalised inverse FFT gives f directly.
#include <hip/hip_ext.h>

#include "common.hpp"
#include "fft.hpp"
#include "launch.hpp"

namespace sdf {

namespace {

using cf = cplx<float>;

constexpr int kSlabBlock = 1024;
// Threads of the slab kernels (spread and inverse slab pass).  The fast slab
// transforms give each thread 8 lines' worth of one radix pass, so N = 64 uses
// 512 threads: more blocks per compute unit instead of one block with half of
// its waves idle in the transforms.  The inverse slab pass writes one argmax
// partial per wave and (rotation, slab).
constexpr int slab_block(int N) { return N == 64 ? 512 : kSlabBlock; }
constexpr int islab_waves(int N) { return slab_block(N) / 64; }
// Threads per line when a block of BLOCK threads transforms LINES lines of
// NZ points (generic sizes): NZ / 8, or else the largest power of two below
// it that lets every line run at once (96 lines of 12 threads exceed 1024
// threads, and a second round of 11 lines leaves most of the block idle).
template <int NZ, int LINES, int BLOCK>
constexpr int fft_tpl() {
    const int t = NZ / 8 < 1 ? 1 : NZ / 8;
    if (LINES * t <= BLOCK) return t;
    int p = 1;
    while (2 * p <= t && LINES * 2 * p <= BLOCK) p *= 2;
    return p;
}
static_assert(fft_tpl<96, 96, 1024>() == 8 && fft_tpl<32, 32, 1024>() == 4, "threads per line");
// Slab transforms of the generic sizes (8, 16, 32, 96): threads per line, and
// the complex row pitch, padded so that the lines one wave transforms along x
// start on different LDS banks.
template <int N>
constexpr int slab_tpl() { return fft_tpl<N, N, slab_block(N)>(); }
template <int N>
constexpr int slab_pitch() { return N + (slab_tpl<N>() < 2 ? 2 : slab_tpl<N>()); }
constexpr int kPencilBlock = 512;
constexpr int kFinishBlock = 256;
constexpr int kPrepBlocks = 64;

template <int N>
constexpr int pencil_width() {
    return N >= 16 ? 16 : N;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// radix schedules selectable per size (threads per line stay N / 8)
template <int N, int P>
struct FusedRadix;
template <> struct FusedRadix<8, 0> { using type = Radices<8>; };
template <> struct FusedRadix<8, 1> { using type = Radices<2, 4>; };
template <> struct FusedRadix<8, 2> { using type = Radices<4, 2>; };
template <> struct FusedRadix<16, 0> { using type = Radices<4, 4>; };
template <> struct FusedRadix<16, 1> { using type = Radices<8, 2>; };
template <> struct FusedRadix<16, 2> { using type = Radices<2, 8>; };
template <> struct FusedRadix<32, 0> { using type = Radices<8, 4>; };
template <> struct FusedRadix<32, 1> { using type = Radices<4, 8>; };
template <> struct FusedRadix<32, 2> { using type = Radices<2, 4, 4>; };
template <> struct FusedRadix<64, 0> { using type = Radices<8, 8>; };
template <> struct FusedRadix<64, 1> { using type = Radices<4, 4, 4>; };
template <> struct FusedRadix<64, 2> { using type = Radices<2, 4, 8>; };
template <> struct FusedRadix<96, 0> { using type = Radices<8, 4, 3>; };
template <> struct FusedRadix<96, 1> { using type = Radices<3, 4, 8>; };
template <> struct FusedRadix<96, 2> { using type = Radices<4, 8, 3>; };
template <> struct FusedRadix<128, 0> { using type = Radices<8, 4, 4>; };
template <> struct FusedRadix<128, 1> { using type = Radices<4, 4, 8>; };
template <> struct FusedRadix<128, 2> { using type = Radices<2, 8, 8>; };

// Copy a row-major N x N complex slab from global memory to LDS rows of
// pitch RS, two entries per 16-byte word: every thread issues all of its
// loads before its first LDS write, so the loads overlap.
template <int N, int RS, int BLOCK>
__device__ __forceinline__ void stage_rows_to_lds(float4* __restrict__ lds, const float4* __restrict__ g) {
    static_assert(N % 2 == 0 && RS % 2 == 0, "two complex entries per 16-byte word");
    constexpr int COUNT = N * N / 2;
    constexpr int PER = (COUNT + BLOCK - 1) / BLOCK;
    float4 r[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int i = threadIdx.x + p * BLOCK;
        if (COUNT % BLOCK == 0 || i < COUNT) r[p] = g[i];
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int i = threadIdx.x + p * BLOCK;
        if (COUNT % BLOCK == 0 || i < COUNT) lds[((2 * i / N) * RS + 2 * i % N) / 2] = r[p];
    }
}

// ------------------------------------------------------------------ rotations
__global__ void rot_desc_kernel(const RotInput* __restrict__ in, int64_t n, FusedRot* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RotInput r = in[i];
    double w = r.q[0], x = r.q[1], y = r.q[2], z = r.q[3];
    const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv;
    x *= inv;
    y *= inv;
    z *= inv;
    const double m[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                         2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
    FusedRot o;
#pragma unroll
    for (int a = 0; a < 9; ++a) o.R[a] = float(m[a]);
    o.job = r.job;
    o.local = r.local;
    if (r.N > 0) {
        // heights of the reflected body nodes -R (k - n_m/2), k in [0, n_m)^3;
        // a slab at centred height zc receives a sample iff |zc - y_z| < 2.
        // The 1e-3 margin covers the FP32 positions the spread kernel forms.
        const double lo = -0.5 * r.n_m, hi = 0.5 * r.n_m - 1.0;
        double zmin = 0.0, zmax = 0.0;
        for (int b = 0; b < 3; ++b) {
            const double a = -m[6 + b];
            zmin += fmin(a * lo, a * hi);
            zmax += fmax(a * lo, a * hi);
        }
        const int zl = int(floor(zmin - 2.0 - 1e-3)), zh = int(ceil(zmax + 2.0 + 1e-3));
        o.zlo = short(zl < -r.N / 2 ? -r.N / 2 : zl);
        o.zhi = short(zh > r.N / 2 - 1 ? r.N / 2 - 1 : zh);
    } else {
        o.zlo = 0;
        o.zhi = 0;
    }
    out[i] = o;
}

// ------------------------------------------------------------------ K0
__global__ __launch_bounds__(256) void cmax_partial_kernel(const FusedJob* __restrict__ jobs,
                                                           float* __restrict__ part) {
    const FusedJob jb = jobs[blockIdx.y];
    const cf* c = static_cast<const cf*>(jb.c);
    const int64_t K = int64_t(jb.n_m) * jb.n_m * (jb.planar ? 1 : jb.n_m);
    float m = 0.f;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < K; i += int64_t(gridDim.x) * 256) {
        const cf v = c[i];
        m = fmaxf(m, fmaxf(fabsf(v.re), fabsf(v.im)));
    }
    for (int off = warpSize / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    __shared__ float wm[4];
    if (threadIdx.x % warpSize == 0) wm[threadIdx.x / warpSize] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
}

// scale = fixed-point units per unit value: |node sum| <= 8 max|c| maps into 2^31
__global__ void cmax_final_kernel(const FusedJob* __restrict__ jobs, const float* __restrict__ part, int nparts) {
    float m = 0.f;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmaxf(m, part[blockIdx.x * nparts + i]);
    for (int off = warpSize / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (threadIdx.x == 0) {
        const float sc = m > 0.f ? 268435456.f / m : 1.f;
        float* out = jobs[blockIdx.x].scale;
        out[0] = sc;
        out[1] = 1.f / sc;
    }
}

// ------------------------------------------------------------------ K1
// Slab layout.  The scatter accumulates into padded rows of 64-bit words:
// row y holds one word per node x, im 2^32 + re of the node's two
// fixed-point sums (one 64-bit LDS add per node instead of two 32-bit ones),
// and 8 pad words, so consecutive rows start 16 banks apart (unpadded rows
// put every row on the same banks and double the scatter's conflict stalls;
// of the pads tried, 8 words was fastest at N = 128).  Positions are stored
// shifted by N / 2 in x and y, which the fitting rule for the rotated body box
// (checked by the ABI for every size) keeps inside [0, N), so no index wraps
// and the 16 stencil addresses of a sample are one base plus constant
// offsets.  The shift multiplies the slab's 2D DFT by (-1)^(kx+ky), removed
// when the slab is written (or folded into the pair-grouped spectrum).  At
// N = 64, 96 and 128 (kRowFft) the complex row that replaces a row after
// conversion keeps entry e at e + e / 16, so that the radix-16 (12) pass
// along x, which writes consecutive entries per lane, does not put the 8
// lanes of a row on the same banks; the other sizes convert to complex rows
// of pitch slab_pitch for the generic transforms.
template <int N>
struct SlabLayout {
    static constexpr bool kFast = N == 64 || N == 128;
    // the spread kernel's register-resident slab transform (8 lanes per
    // row): the fast sizes and N = 96 (radix 12 x 8, row-major store)
    static constexpr bool kRowFft = kFast || N == 96;
    static constexpr int kRowInts = 2 * N + 16;      // 32-bit words per accumulation row
    static constexpr int kInts = N * kRowInts;       // >= 2 N N: room for the complex slab
    static constexpr int kRowCf = kRowInts / 2;      // 64-bit node words per row = complex stride (fast)
    static constexpr int kShift = N / 2;
    static_assert(!kRowFft || kRowCf >= N + N / 16, "a converted row (N entries and N / 16 gaps) fits its row");
};

__device__ __forceinline__ int fixed_rpi(float v) {
    // round to nearest (halves up) in one instruction
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// Add a 4 x 4 stencil of fixed-point values (re in vr, im in vi, index
// 4 b + a for node (ix + a, iy + b)) to the slab's node words.  A word gets
// im 2^32 + re with re sign-extended: its high half is im minus the borrow
// of a negative re.
template <int N>
__device__ __forceinline__ void flush_stencil(int* __restrict__ acc, int ix, int iy, const int vr[16],
                                              const int vi[16]) {
    using L = SlabLayout<N>;
    unsigned long long* acc64 = reinterpret_cast<unsigned long long*>(acc);
    const int base = int(__umul24(unsigned(iy + L::kShift), unsigned(L::kRowCf))) + ix + L::kShift;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int re = vr[4 * b + a], im = vi[4 * b + a];
            const unsigned long long v =
                (static_cast<unsigned long long>(unsigned(im + (re >> 31))) << 32) | unsigned(re);
            atomicAdd(acc64 + base + b * L::kRowCf + a, v);
        }
    }
}

// The (re, im) sums of a node from its 64-bit word: the word holds
// im 2^32 + re exactly (modulo 2^64), so with both sums in int32 range the
// low half is re and the high half is im minus the borrow of a negative re.
__device__ __forceinline__ void unpack_node(unsigned long long s, int& re, int& im) {
    re = int(unsigned(s));
    im = int(unsigned(s >> 32)) - (re >> 31);
}

// Spread the samples of one (rotation, z-slab) item into the slab's node words.
// lines of a (rotation, slab) item compacted per round; the list of their
// runs lives in LDS next to the slab
constexpr int kLineChunk = 4096;

template <int N>
__device__ __forceinline__ void spread_item(int* __restrict__ acc, const FusedRot& fr, const cf* __restrict__ c,
                                            int n_m, float S, int z, bool planar, int* __restrict__ list,
                                            int* __restrict__ nlist) {
    constexpr int B = slab_block(N);
    // reflected rotation: positions y_k = Rp (k - n_m / 2), Rp = -R
    float Rp[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) Rp[a] = -fr.R[a];
    const float half = 0.5f * float(n_m);
    if (planar) {
        const int K = n_m * n_m;
        for (int k = threadIdx.x; k < K; k += B) {
            const cf ck = gload(c, k);
            const float bx = float(k % n_m) - half, by = float(k / n_m) - half;
            const float yx = Rp[0] * bx + Rp[1] * by;
            const float yy = Rp[3] * bx + Rp[4] * by;
            const float fx = floorf(yx), fy = floorf(yy);
            float wx[4], wy[4], xr[4], xi[4];
            bspline3_weights(yx - fx, wx);
            bspline3_weights(yy - fy, wy);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                xr[a] = ck.re * S * wx[a];
                xi[a] = ck.im * S * wx[a];
            }
            int vr[16], vi[16];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    vr[4 * b + a] = fixed_rpi(xr[a] * wy[b]);
                    vi[4 * b + a] = fixed_rpi(xi[a] * wy[b]);
                }
            }
            flush_stencil<N>(acc, int(fx) - 1, int(fy) - 1, vr, vi);
        }
        return;
    }
    // Walk body lines along the axis ax most aligned with z: for each
    // (k_b1, k_b2) the samples y(ka) = y0 + ka d (d = column ax of the
    // reflected rotation) cross the slab support |z - y_z| < 2 for a short
    // run of ka.  Only about half of the lines reach a given slab, so the
    // lines are first compacted: every thread finds the runs of its lines
    // and the lines with a non-empty run are appended to an LDS list (each
    // wave appends its lines in lane order), then the threads take the
    // listed lines and spread their runs, the next coefficient fetched one
    // step ahead.  Lines are enumerated in 16 x 16 blocks by four waves: a
    // wave covers 8 rows of the block (b2) and every other line along b1
    // (the axis most aligned with x), offset by one on alternate rows, so the
    // lanes of a wave spread nearby lines whose samples sit at nearby
    // heights; the stride keeps two lanes from adding to the same LDS word in
    // one instruction, which the LDS serialises (lanes on consecutive lines
    // made the kernel 12% slower), and the row offset spreads the lanes over
    // odd and even banks.  The order in which waves append does not matter:
    // the integer sums do not depend on it.
    int ax = 0;
    float best = fabsf(Rp[6]);
    if (fabsf(Rp[7]) > best) { ax = 1; best = fabsf(Rp[7]); }
    if (fabsf(Rp[8]) > best) { ax = 2; }
    int b1 = ax == 0 ? 1 : 0;
    int b2 = ax == 2 ? 1 : 2;
    if (fabsf(Rp[b2]) > fabsf(Rp[b1])) { const int t = b1; b1 = b2; b2 = t; }
    const float dx = Rp[ax], dy = Rp[3 + ax], dzs = Rp[6 + ax];
    const float inv_dz = 1.f / dzs;
    const int kstride[3] = {1, n_m, n_m * n_m};
    const int sax = kstride[ax];
    const float zc = float(z < N / 2 ? z : z - N);  // centred image of this slab
    const int pairs = n_m * n_m;
    const bool blocks16 = (n_m & 15) == 0;
    const int nb16 = n_m >> 4;
    const float u0 = -half;
    const int lane = threadIdx.x & 63;
    // the coefficients through a buffer descriptor: a 32-bit offset stepped
    // along the line, and the read one past a run's last sample needs no
    // branch (its value is not used; past the end of c it reads zeros)
    const __amdgpu_buffer_rsrc_t crs = buffer_rsrc(c, uint32_t(pairs) * uint32_t(n_m) * uint32_t(sizeof(cf)));
    for (int c0 = 0; c0 < pairs; c0 += kLineChunk) {
        if (threadIdx.x == 0) *nlist = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kLineChunk / B; ++r) {
            const int pidx = c0 + threadIdx.x + r * B;
            int entry = 0;
            bool ne = false;
            if (pidx < pairs) {
                int i1, i2;
                if (blocks16) {
                    const int w = pidx >> 6, l = pidx & 63;
                    const int blk = w >> 2, k = w & 3;
                    const int row = (l >> 3) + 8 * (k >> 1);  // 0 .. 15 within the block
                    i2 = (blk / nb16) * 16 + row;
                    i1 = (blk % nb16) * 16 + 2 * (l & 7) + ((row + k) & 1);
                } else {
                    i1 = pidx % n_m;
                    i2 = pidx / n_m;
                }
                const float u1 = float(i1) - half, u2 = float(i2) - half;
                const float y0z = Rp[6 + b1] * u1 + Rp[6 + b2] * u2 + dzs * u0;
                float lo_f = (zc - 2.f - y0z) * inv_dz, hi_f = (zc + 2.f - y0z) * inv_dz;
                if (lo_f > hi_f) { const float t = lo_f; lo_f = hi_f; hi_f = t; }
                // samples strictly inside (lo_f, hi_f); a 1e-3 margin keeps any
                // sample that rounding could place inside, and the support test
                // below decides
                int lo = int(floorf(lo_f + 0.999f)), hi = int(ceilf(hi_f - 0.999f));
                lo = lo < 0 ? 0 : lo;
                hi = hi > n_m - 1 ? n_m - 1 : hi;
                ne = lo <= hi;
                entry = i1 | (i2 << 7) | (lo << 14) | (hi << 21);
            }
            const uint64_t m = __ballot(ne);
            if (m != 0ull) {  // uniform across the wave
                int wbase = 0;
                if (lane == 0) wbase = atomicAdd(nlist, int(__popcll(m)));
                wbase = __shfl(wbase, 0);
                if (ne) list[wbase + int(__popcll(m & ((1ull << lane) - 1ull)))] = entry;
            }
        }
        __syncthreads();
        const int nl = *nlist;
        for (int e = threadIdx.x; e < nl; e += B) {
            const int entry = list[e];
            const int i1 = entry & 127, i2 = (entry >> 7) & 127, lo = (entry >> 14) & 127, hi = entry >> 21;
            const float u1 = float(i1) - half, u2 = float(i2) - half;
            const float y0x = Rp[b1] * u1 + Rp[b2] * u2 + dx * u0;
            const float y0y = Rp[3 + b1] * u1 + Rp[3 + b2] * u2 + dy * u0;
            const float y0z = Rp[6 + b1] * u1 + Rp[6 + b2] * u2 + dzs * u0;
            const int k0 = i1 * kstride[b1] + i2 * kstride[b2];
            // the three weight factors are computed six times too large (the
            // B-spline's 1/6 left out) and S6 = S / 216 restores them
            const float S6 = S * (1.f / 216.f);
            uint32_t coff = uint32_t(k0 + lo * sax) * uint32_t(sizeof(cf));
            const uint32_t cstep = uint32_t(sax) * uint32_t(sizeof(cf));
            cf cnext = buffer_load_cf(crs, coff, 0);
            for (int ka = lo; ka <= hi; ++ka) {
                const cf ck = cnext;
                coff += cstep;
                cnext = buffer_load_cf(crs, coff, 0);
                const float fk = float(ka);
                const float yz = y0z + fk * dzs;
                const float ad = fabsf(zc - yz);
                if (!(ad < 2.f)) continue;
                const float yx = y0x + fk * dx;
                const float yy = y0y + fk * dy;
                // 6 beta(ad) = (2 - ad)^3 - 4 (1 - ad)^3_+, without a branch
                const float bz = 2.f - ad, az = fmaxf(1.f - ad, 0.f);
                const float wz6 = bz * bz * bz - 4.f * (az * az * az);
                const float sw = wz6 * S6;
                const float fx = floorf(yx), fy = floorf(yy);
                float wx[4], wy[4], xr[4], xi[4];
                bspline3_weights6(yx - fx, wx);
                bspline3_weights6(yy - fy, wy);
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    xr[a] = ck.re * sw * wx[a];
                    xi[a] = ck.im * sw * wx[a];
                }
                int vr[16], vi[16];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        vr[4 * b + a] = fixed_rpi(xr[a] * wy[b]);
                        vi[4 * b + a] = fixed_rpi(xi[a] * wy[b]);
                    }
                }
                flush_stencil<N>(acc, int(fx) - 1, int(fy) - 1, vr, vi);
            }
        }
        __syncthreads();  // the list is rewritten by the next chunk
    }
}

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Forward 2D DFT of the padded slab (N = 8 R1, R1 = 8, 12 or 16) and its store.
// Along x, 8 consecutive lanes own one row for both passes (radix R1, then
// radix 8 with twiddles), so the x transform needs no block barrier: one
// wave's LDS operations complete in issue order.  The first pass reads the
// node words and converts.  Along y, pass C (radix R1) is split by a
// barrier between its reads and writes; pass D (radix 8) reads, writes the
// result to global memory with the (-1)^(kx+ky) shift correction, and
// clears the LDS words it read for the next item.
template <int N>
__device__ __forceinline__ void slab_fft_store_fast(int* __restrict__ acc, const cf* __restrict__ tw, float inv,
                                                    cf* __restrict__ out, bool grouped, int z) {
    using L = SlabLayout<N>;
    constexpr int R1 = N / 8;
    constexpr int NB = N / 8;   // radix-8 butterflies per line
    constexpr int RS = L::kRowCf;
    auto px = [](int e) { return e + (e >> 4); };
    cf* slab = reinterpret_cast<cf*>(acc);
    // opaque copy of the thread index: keeps the compiler from hoisting this
    // phase's ~60 address registers out of the item loop, where they would
    // stay live through the scatter and spill
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    {
        const int y = t / 8, j = t % 8;
        if (y < N) {
            cf v[R1];
            int any = 0;
#pragma unroll
            for (int r = 0; r < R1; ++r) {
                const int x = j + 8 * r;
                int a, b;
                unpack_node(reinterpret_cast<const unsigned long long*>(acc)[y * L::kRowCf + x], a, b);
                any |= a | b;
                v[r] = mk(float(a) * inv, float(b) * inv);
            }
            // A row the scatter did not touch transforms to zeros, which the
            // LDS already holds (integer 0 and float +0 share their bits):
            // the 8 lanes of such a row skip both x passes.
            const uint64_t touched = __ballot(any != 0);
            if (((touched >> ((threadIdx.x & 63) & ~7)) & 0xffull) == 0) goto x_done;
            compiler_fence();
            dftR<float, -1, R1>(v);
#pragma unroll
            for (int r = 0; r < R1; ++r) slab[y * RS + px(j * R1 + r)] = v[r];
            compiler_fence();
#pragma unroll
            for (int m = 0; m < (NB + 7) / 8; ++m) {
                const int jj = j + 8 * m;  // k = jj
                if (NB % 8 != 0 && jj >= NB) break;  // R1 = 12: lanes 0-3 take a second butterfly
                cf u[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) u[r] = slab[y * RS + px(jj + NB * r)];
#pragma unroll
                for (int r = 1; r < 8; ++r) u[r] = u[r] * tw[r * jj];
                dft8<float, -1>(u);
#pragma unroll
                for (int r = 0; r < 8; ++r) slab[y * RS + px(jj + NB * r)] = u[r];
            }
        }
    }
x_done:
    __syncthreads();
    const int x = t % N, jb = t / N;
    const bool on = jb < 8;
    {
        cf v[R1];
        if (on) {
#pragma unroll
            for (int r = 0; r < R1; ++r) v[r] = slab[(jb + 8 * r) * RS + px(x)];
            dftR<float, -1, R1>(v);
        }
        __syncthreads();
        if (on) {
#pragma unroll
            for (int r = 0; r < R1; ++r) slab[(jb * R1 + r) * RS + px(x)] = v[r];
        }
        __syncthreads();
    }
    if (on) {
#pragma unroll
        for (int m = 0; m < (NB + 7) / 8; ++m) {
            const int jj = jb + 8 * m;
            if (NB % 8 != 0 && jj >= NB) break;
            cf u[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) u[r] = slab[(jj + NB * r) * RS + px(x)];
#pragma unroll
            for (int r = 1; r < 8; ++r) u[r] = u[r] * tw[r * jj];
            dft8<float, -1>(u);
            // 32-bit element offsets from a uniform base: the rotation's grid
            // in column tiles (3D) or the item's slab (planar)
            const unsigned col = unsigned(grouped ? tile_index<N>(z, jj, col_pos<N>(x)) : jj * N + x);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int ky = jj + NB * r;
                // the (-1)^(kx + ky) of the N / 2 shift: folded into the
                // pair-grouped spectrum, applied here otherwise (planar)
                const cf v = (!grouped && ((x + ky) & 1)) ? mk(-u[r].re, -u[r].im) : u[r];
                out[col + unsigned(NB * r * N * (grouped ? N : 1))] = v;
                slab[ky * RS + px(x)] = mk(0.f, 0.f);
                if (x < N / 16) slab[ky * RS + 17 * x + 16] = mk(0.f, 0.f);  // the gap entries
            }
        }
    }
}

// Work item = (z-slab, rotation), z fastest.
template <int N, int P>
__global__ __launch_bounds__(slab_block(N)) void spread_slab_kernel(const FusedRot* __restrict__ rots,
                                                                     const FusedJob* __restrict__ jobs, int n_rot,
                                                                     int planar, cf* __restrict__ slabs) {
    constexpr int B = slab_block(N);
    using L = SlabLayout<N>;
    using Plan = typename FusedRadix<N, P>::type;
    __shared__ __align__(16) int acc[L::kInts];
    __shared__ cf tw[N];
    __shared__ int list[kLineChunk];  // packed (i1, i2, lo, hi) of the lines that reach the slab
    __shared__ int nlist;
    static_assert(sizeof(int) * (L::kInts + kLineChunk + 1) + sizeof(cf) * N <= 160 * 1024,
                  "one block's LDS must fit the 160 KiB of a compute unit");
    fill_twiddles<float, N>(tw);
    const int nz = planar ? 1 : N;
    const int items = nz * n_rot;
    if constexpr (L::kRowFft) {
        for (int i = threadIdx.x; i < L::kInts; i += B) acc[i] = 0;  // later items clear as they store
    }
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        // The scatter work of a slab follows the body's cross-section at its
        // height, largest near z = 0.  With the grid a multiple of nz a
        // block would see the same z for every rotation; offsetting z by
        // 53 (odd) per rotation gives every block a spread of heights.
        const int rot = item / nz;
        const int z = (item % nz + 53 * (rot % nz)) % nz;
        const FusedRot fr = rots[rot];
        const int zc = z < N / 2 ? z : z - N;
        if (nz > 1 && (zc < fr.zlo || zc > fr.zhi)) continue;  // uniform: the slab is zero and is not written
        const FusedJob jb = jobs[fr.job];
        __syncthreads();  // previous item done with the slab
        if constexpr (!L::kRowFft) {
            for (int i = threadIdx.x; i < L::kInts; i += B) acc[i] = 0;
            __syncthreads();
        }
        spread_item<N>(acc, fr, static_cast<const cf*>(jb.c), jb.n_m, jb.scale[0], z, planar != 0, list, &nlist);
        __syncthreads();
        cf* out = slabs + (int64_t(rot) * nz + z) * N * N;
        const float inv = jb.scale[1];
        if constexpr (L::kFast) {
            // 3D grids: the rotation's column tiles; planar: the slab
            slab_fft_store_fast<N>(acc, tw, inv, planar ? out : slabs + int64_t(rot) * nz * N * N, planar == 0, z);
        } else if constexpr (L::kRowFft) {
            slab_fft_store_fast<N>(acc, tw, inv, out, false, z);  // row-major slab
        } else {
            // node words -> padded complex rows, in place: read everything, then write
            constexpr int TPL = slab_tpl<N>(), RS = slab_pitch<N>();
            static_assert(2 * N * RS <= L::kInts, "the complex slab must fit the node words");
            cf* slab = reinterpret_cast<cf*>(acc);
            constexpr int PER = (N * N + B - 1) / B;
            cf v[PER];
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int i = threadIdx.x + p * B;
                if ((N * N) % B == 0 || i < N * N) {
                    int a, b;
                    unpack_node(reinterpret_cast<const unsigned long long*>(acc)[(i / N) * L::kRowCf + i % N], a, b);
                    v[p] = mk(float(a) * inv, float(b) * inv);
                }
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int i = threadIdx.x + p * B;
                if ((N * N) % B == 0 || i < N * N) slab[(i / N) * RS + i % N] = v[p];
            }
            __syncthreads();
            lds_fft_lines<float, N, -1, false, Plan, TPL>(slab, 1, RS, N, tw);  // along x
            lds_fft_lines<float, N, -1, true, Plan, TPL>(slab, RS, 1, N, tw);   // along y
            // the (-1)^(kx + ky) of the N / 2 shift
            for (int i = threadIdx.x; i < N * N; i += B) {
                const cf v = slab[(i / N) * RS + i % N];
                out[i] = ((i % N + i / N) & 1) ? mk(-v.re, -v.im) : v;
            }
        }
    }
}

// ------------------------------------------------------------------ K2
// z transform of LINES lines of NZ = 8 R1 points held at buf[kz * NL + l]
// (generic pencils; R1 = 12): thread (l, jb), jb < 8, takes the points
// kz = jb + 8 r into registers for a radix-R1 DFT, then runs radix 8 with
// twiddles on rows jj + R1 r (jj = jb, and jb + 8 while below R1), which no
// other thread touches; natural order out.  Two barriers instead of the
// Stockham passes' six per round.  Every thread of the block calls it.
template <int NZ, int S, int NL, int LINES, int BLOCK>
__device__ __forceinline__ void zfft_lines_r8(cf* __restrict__ buf, const cf* __restrict__ tw) {
    constexpr int R1 = NZ / 8, NB = NZ / 8;
    static_assert(NZ % 8 == 0 && LINES <= NL && NL * 8 <= BLOCK, "one thread per (line, jb)");
    const int l = int(threadIdx.x) % NL, jb = int(threadIdx.x) / NL;
    const bool on = l < LINES && jb < 8;
    cf v[R1];
    if (on) {
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = buf[(jb + 8 * r) * NL + l];
        dftR<float, S, R1>(v);
    }
    __syncthreads();
    if (on) {
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[(jb * R1 + r) * NL + l] = v[r];
    }
    __syncthreads();
    if (on) {
#pragma unroll
        for (int m = 0; m < (NB + 7) / 8; ++m) {
            const int jj = jb + 8 * m;
            if (NB % 8 != 0 && jj >= NB) break;
            cf u[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) u[r] = buf[(jj + NB * r) * NL + l];
#pragma unroll
            for (int r = 1; r < 8; ++r) u[r] = u[r] * (S < 0 ? tw[r * jj] : conj(tw[r * jj]));
            dft8<float, S>(u);
#pragma unroll
            for (int r = 0; r < 8; ++r) buf[(jj + NB * r) * NL + l] = u[r];
        }
    }
    __syncthreads();
}
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

// pair-grouped layout: rows ky = 0 .. N/2 (each with its partner row -ky),
// every aligned 16-position block
// (instantiated for every size, used only for N = 64 and 128)
template <int N>
constexpr int pencil_blocks16() {
    return N >= 16 ? N / 16 : 1;
}
template <int N>
constexpr int pencil_jobs_grouped() {
    return (N / 2 + 1) * pencil_blocks16<N>();
}
template <int N>
__device__ __forceinline__ PencilJob pencil_job_grouped(int j) {
    return PencilJob{j / pencil_blocks16<N>(), (j % pencil_blocks16<N>()) * 16};
}

// Rotation (within its group of GR) of the line group q = l / W, for lines
// l = ((r & 1) GR + (r >> 1) 2 + tile) W + cc: groups 2 p and 2 p + 1 (the
// two tiles) belong to the same rotation.
template <int GR>
__device__ __forceinline__ int pencil_group_rot(int q) {
    return 2 * ((q % GR) / 2) + q / GR;
}

// Pass-A chunk ch of an item (pencil job, rotations g0 ..): the 2 W lines of
// one rotation (both tiles) at two values of j, with the R1 values
// kz = j + 8 r of each line.  The rotation, its slab range and the buffer
// descriptor are wave-uniform; slabs outside the rotation's range were never
// written and read as zeros through out-of-range offsets, as do rotations
// past n_rot.
template <int N, int GR>
struct PencilChunk {
    static constexpr int W = pencil_width<N>();
    static constexpr int NL = 2 * W * GR;
    static constexpr int R1 = N / 8;
    static constexpr int kChunks = NL * 8 / 64;
    static_assert(NL * 8 % 64 == 0 && 2 * W == 32, "pass A chunks are 32 lines x 2 values of j");
    int l, j, cc, tt;
    __device__ __forceinline__ PencilChunk(int ch, int lane) {
        const int qp = ch % (NL / 32), jg = ch / (NL / 32);
        l = 32 * qp + (lane & 31);
        j = 2 * jg + (lane >> 5);
        cc = l % W;
        tt = (l / W) % 2;
    }
    __device__ __forceinline__ static int rot_in_group(int ch) { return pencil_group_rot<GR>(2 * (ch % (NL / 32))); }
};

// ALL: every kz is present (transformed spectra rather than spread slabs)
template <int N, int GR, bool ALL = false>
__device__ __forceinline__ void pencil_load_chunk(const cf* __restrict__ slabs, const FusedRot* __restrict__ rots,
                                                  int n_rot, const PencilJob job, int g0, int ch, int lane,
                                                  cf (&v)[N / 8]) {
    using C = PencilChunk<N, GR>;
    constexpr int64_t G = int64_t(N) * N * N;
    constexpr uint32_t kGridBytes = uint32_t(G * sizeof(cf));
    static_assert(G * sizeof(cf) < (int64_t(1) << 31), "buffer offsets are 32-bit");
    const C c(ch, lane);
    const int rot = uniform(g0 + C::rot_in_group(ch));
    if (rot < n_rot) {
        const int zlo = ALL ? -N / 2 : uniform(rots[rot].zlo), span = ALL ? N - 1 : uniform(rots[rot].zhi) - zlo;
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(slabs + int64_t(rot) * G, kGridBytes);
        const int ky = c.tt ? (N - job.ky) % N : job.ky;
        const uint32_t vo = uint32_t(tile_index<N>(c.j, ky, job.x0 + c.cc) * int(sizeof(cf)));
        const int d = c.j - zlo;
#pragma unroll
        for (int r = 0; r < C::R1; ++r) {
            // centred height of kz = j + 8 r, minus zlo
            const int dz = d + 8 * r - (8 * r < N / 2 ? 0 : N);
            const bool reached = unsigned(dz) <= unsigned(span);
            v[r] = buffer_load_cf(rs, reached ? vo : kBufferNone, uint32_t(8 * r * 16 * sizeof(cf)));
        }
    } else {
#pragma unroll
        for (int r = 0; r < C::R1; ++r) v[r] = mk(0.f, 0.f);
    }
}

// Fast pencil pass for NZ = N = 8 R1 (R1 = 8 or 16).  LDS holds the NL
// lines of the item at row stride NL + 8 (element kz of line l at
// kz (NL + 8) + l).
//  A  forward radix-R1 pass along z.  With GR = 2 the item's raw columns are
//     already in LDS (rows j R1 + r of line l hold kz = j + 8 r), loaded
//     during the previous item's inverse passes; with GR = 4 each wave loads
//     its chunks here;
//  B  forward radix-8 pass in place, times the fixed spectrum;
//  F  Hermitian folding in place: the unit (pair, column, kz) reads the k
//     lines a0, b0 at kz and the -k lines a1, b1 at -kz and writes Z to a0
//     at kz and a1 at -kz, positions no other unit touches;
//  I  inverse radix-R1 and radix-8 passes over the Z lines, 8 lines per
//     wave, the last pass writing global memory.  With GR = 2 the next
//     item's columns are loaded meanwhile and written to LDS after a barrier:
//     at N = 128 every wave loads one chunk, the 4 line groups' waves run the
//     first pass, and after a barrier the second pass's two butterfly sets of
//     each line group go to its wave and to one of the other 4; otherwise the
//     line groups' waves run both passes (no block barrier between them)
//     while the other 4 waves load two chunks each.
// The spectrum values of a thread's pass-B units (GR = 2: two units of 8
// values) are kept in registers, and consecutive items of a block that share
// the pencil job and the spectra reuse them.
// GR = 2 with 16-column tiles: the Z lines form GR W / 8 = 4 line groups of
// 8 lines, one per wave of the first 4, and the next item has 8 chunks
template <int N, int GR>
constexpr bool pencil_pipe() {
    if constexpr (pencil_width<N>() != 16 || GR != 2) {
        return false;
    } else {
        constexpr int IW = GR * pencil_width<N>() / 8;
        return IW < kPencilBlock / 64 && PencilChunk<N, GR>::kChunks == 2 * (kPencilBlock / 64 - IW);
    }
}

template <int N, int GR>
struct PencilSpec {
    static constexpr int NL = 2 * pencil_width<N>() * GR;
    static constexpr int NB = N / 8;
    static constexpr int PB = (NL * NB + kPencilBlock - 1) / kPencilBlock;
    static constexpr bool kKeep = GR == 2 && PB * kPencilBlock == NL * NB;
    static constexpr int kRows = kKeep ? PB : 1;
    // waves that run the inverse passes; the others load ahead when PIPE
    static constexpr int IW = GR * pencil_width<N>() / 8;
    static constexpr bool kPipe = pencil_pipe<N, GR>();
};

// next item of the block, for the loads ahead
struct PencilNext {
    PencilJob job;
    int g0;
    bool valid;
};

// raw columns into LDS: for the forward pass A (row j R1 + r holds
// kz = j + 8 r), or NATURAL: transformed spectra at row kz, times the fold's
// factor 1/2
template <int N, int GR, bool NATURAL = false>
__device__ __forceinline__ void pencil_store_raw(cf* __restrict__ buf, int ch, int lane, const cf (&v)[N / 8]) {
    using C = PencilChunk<N, GR>;
    constexpr int NLP = C::NL + 8;
    const C c(ch, lane);
#pragma unroll
    for (int r = 0; r < C::R1; ++r) {
        if constexpr (NATURAL)
            buf[(c.j + 8 * r) * NLP + c.l] = v[r] * 0.5f;
        else
            buf[(c.j * C::R1 + r) * NLP + c.l] = v[r];
    }
}

// MODES: the input is already transformed along z and multiplied by the
// spectrum (column tiles, every kz): passes A and B are skipped, the loader
// waves put the next item's values straight into their rows
template <int N, int GR, bool MODES = false>
__device__ __forceinline__ void pencil_item_fast(int n_rot, const FusedRot* __restrict__ rots,
                                                 const cf* __restrict__ slabs, cf* __restrict__ packed,
                                                 cf* __restrict__ buf, const cf* __restrict__ tw,
                                                 const cf* const* spec_of, const PencilJob job, int g0,
                                                 const PencilNext nx, cf (&spre)[PencilSpec<N, GR>::kRows][8],
                                                 bool reload) {
    using PS = PencilSpec<N, GR>;
    using C = PencilChunk<N, GR>;
    constexpr int W = pencil_width<N>();
    constexpr int NL = 2 * W * GR;
    constexpr int NLP = NL + 8;
    constexpr int R1 = N / 8;
    constexpr int NB = N / 8;
    constexpr int64_t G = int64_t(N) * N * N;
    constexpr uint32_t kGridBytes = uint32_t(G * sizeof(cf));
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int lane = t & 63, wave = uniform(t >> 6);
    const int kyt[2] = {job.ky, (N - job.ky) % N};
    // both tiles cover positions x0 .. x0 + 15 of the pair-grouped order; the
    // partner of position x0 + cc is x0 + (cc ^ 8), or itself for kx = 0, N/2
    auto kx_of = [&](int, int cc) { return job.x0 + cc; };
    auto partner = [&](int cc) { return (job.x0 == 0 && (cc & 7) == 0) ? cc : (cc ^ 8); };
    constexpr int PB = PS::PB;
    constexpr bool kPre = PS::kKeep;
    auto spec_at = [&](int b, int r) {
        const int l = b % NL, jj = b / NL;
        const int cc = l % W, tt = (l / W) % 2;
        const cf* sp = spec_of[pencil_group_rot<GR>(l / W)];
        return sp ? gload(sp, tile_index<N>(jj + NB * r, kyt[tt], kx_of(tt, cc))) : mk(0.f, 0.f);
    };
    static_assert(!MODES || PS::kPipe, "transformed input comes through the loader waves");
    if constexpr (kPre && !MODES) {
        if (reload) {
#pragma unroll
            for (int m = 0; m < PB; ++m)
#pragma unroll
                for (int r = 0; r < 8; ++r) spre[m][r] = spec_at(t + m * kPencilBlock, r);
        }
    }
    // ---- A
    for (int ch = wave; !MODES && ch < C::kChunks; ch += kPencilBlock / 64) {
        const C c(ch, lane);
        cf v[R1];
        if constexpr (PS::kPipe) {
#pragma unroll
            for (int r = 0; r < R1; ++r) v[r] = buf[(c.j * R1 + r) * NLP + c.l];
        } else {
            pencil_load_chunk<N, GR>(slabs, rots, n_rot, job, g0, ch, lane, v);
        }
        dftR<float, -1, R1>(v);
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[(c.j * R1 + r) * NLP + c.l] = v[r];
    }
    __syncthreads();
    // ---- B (the grouped spectrum carries the fold's factor 1/2)
#pragma unroll
    for (int m = 0; m < (MODES ? 0 : PB); ++m) {
        const int b = t + m * kPencilBlock;
        if (!kPre && b >= NL * NB) break;
        const int l = b % NL, jj = b / NL;
        cf u[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) u[r] = buf[(jj + NB * r) * NLP + l];
#pragma unroll
        for (int r = 1; r < 8; ++r) u[r] = u[r] * tw[r * jj];
        dft8<float, -1>(u);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const cf sv = kPre ? spre[kPre ? m : 0][r] : spec_at(b, r);
            buf[(jj + NB * r) * NLP + l] = u[r] * sv;
        }
    }
    __syncthreads();
    // ---- F: unit (pair p, column cc, kz); a thread keeps cc and walks kz in
    // steps of KS, so its rows sit at constant offsets from two bases
    {
        constexpr int KS = kPencilBlock / W;  // kz step between a thread's units
        constexpr int NM = N / KS;             // units per pair and thread
        static_assert(kPencilBlock % W == 0 && N % KS == 0, "fold units");
        const int cc = t % W, kz0 = t / W;
        const int pc = partner(cc);
        const int mk0 = kz0 == 0 ? 0 : N - kz0;  // -kz0 mod N
#pragma unroll
        for (int p = 0; p < GR / 2; ++p) {
            const int a0 = (2 * p) * W + cc, a1 = (2 * p + 1) * W + pc;
            const int b0 = (GR + 2 * p) * W + cc, b1 = (GR + 2 * p + 1) * W + pc;
#pragma unroll
            for (int s = 0; s < NM; ++s) {
                const int kz = kz0 + KS * s;
                const int mkz = s == 0 ? mk0 : N - kz0 - KS * s;
                const cf ya0 = buf[kz * NLP + a0], ya1 = buf[mkz * NLP + a1];
                const cf yb0 = buf[kz * NLP + b0], yb1 = buf[mkz * NLP + b1];
                const cf ha = ya0 + conj(ya1);
                const cf hb = yb0 + conj(yb1);
                buf[kz * NLP + a0] = mk(ha.re - hb.im, ha.im + hb.re);
                buf[mkz * NLP + a1] = mk(ha.re + hb.im, hb.re - ha.im);
            }
        }
    }
    __syncthreads();
    // ---- I: Z lines are lines [0, GR W); wave w takes lines 8 w .. 8 w + 7,
    // which lie in one (pair, tile) group, so the stores go through one
    // wave-uniform descriptor.  The other waves load the next item.
    cf pre[PS::kPipe ? 2 : 1][R1];
    const bool loader = PS::kPipe && wave >= PS::IW && nx.valid;
    // first inverse pass (radix R1) of the lines of wave wv, in place
    auto inv_first = [&](int wv) {
        const int l = wv * 8 + (lane & 7), j = lane >> 3;
        cf v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = buf[(j + 8 * r) * NLP + l];
        compiler_fence();
        dftR<float, 1, R1>(v);
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[(j * R1 + r) * NLP + l] = v[r];
        compiler_fence();
    };
    // second inverse pass (radix 8), butterflies m0, m0 + ms, .. of the lines
    // of wave wv, written to global memory
    auto inv_last = [&](int wv, int m0, int ms) {
        const int l = wv * 8 + (lane & 7), j = lane >> 3;
        const int cc = l % W, q = (wv * 8) / W, p = q / 2, tt = q % 2;
        const int pair = g0 / 2 + p;
        const bool store = pair < (n_rot + 1) / 2;
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(packed + int64_t(store ? pair : 0) * G, kGridBytes);
#pragma unroll
        for (int m = m0; m < NB / 8; m += ms) {
            const int jj = j + 8 * m;
            cf uu[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) uu[r] = buf[(jj + NB * r) * NLP + l];
#pragma unroll
            for (int r = 1; r < 8; ++r) uu[r] = uu[r] * conj(tw[r * jj]);
            dft8<float, 1>(uu);
            if (store) {
                const uint32_t vo = uint32_t(((jj * N + kyt[tt]) * N + kx_of(tt, cc)) * int(sizeof(cf)));
#pragma unroll
                for (int r = 0; r < 8; ++r) buffer_store_cf(uu[r], rs, vo, uint32_t(NB * r * N * N * sizeof(cf)));
            }
        }
    };
    if constexpr (PS::kPipe && NB / 8 == 2) {
        // every wave loads one chunk of the next item; the line groups' waves
        // run the first pass, and the second pass's two butterfly sets are
        // split between a line group's wave and one of the others.  The loads
        // stay in flight through the barriers (they wait for LDS operations
        // only)
        if (nx.valid) pencil_load_chunk<N, GR, MODES>(slabs, rots, n_rot, nx.job, nx.g0, wave, lane, pre[0]);
        if (wave < PS::IW) inv_first(wave);
        __syncthreads();
        inv_last(wave % PS::IW, wave < PS::IW ? 0 : 1, 2);
        __syncthreads();  // the inverse passes are done with buf
        if (nx.valid) pencil_store_raw<N, GR, MODES>(buf, wave, lane, pre[0]);
        return;
    } else if (!PS::kPipe || wave < PS::IW) {
        for (int wv = wave; wv < PS::IW; wv += kPencilBlock / 64) {
            inv_first(wv);
            inv_last(wv, 0, 1);
        }
    } else if (loader) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
            pencil_load_chunk<N, GR, MODES>(slabs, rots, n_rot, nx.job, nx.g0, 2 * (wave - PS::IW) + k, lane,
                                            pre[k]);
    }
    if constexpr (PS::kPipe) {
        __syncthreads();  // the inverse passes are done with buf
        if (loader) {
#pragma unroll
            for (int k = 0; k < 2; ++k) pencil_store_raw<N, GR, MODES>(buf, 2 * (wave - PS::IW) + k, lane, pre[k]);
        }
    }
}

// Work item = (pencil tile pair, group of GR rotations).  NZ = N (3D) or 1 (planar).
template <int N, int NZ, int GR, int P>
__global__ __launch_bounds__(kPencilBlock, 4) void pencil_kernel(const FusedRot* __restrict__ rots,
                                                              const FusedJob* __restrict__ jobs, int n_rot,
                                                              const cf* __restrict__ slabs,
                                                              cf* __restrict__ packed) {
    using Plan = typename FusedRadix<(NZ > 1 ? NZ : 8), P>::type;
    constexpr int W = pencil_width<N>();
    constexpr int NL = 2 * W * GR;  // lines: (rotation, tile, column)
    constexpr bool kFast = NZ == N && SlabLayout<N>::kFast;
    __shared__ cf buf[kFast ? NZ * (NL + 8) : NZ * NL];
    // generic sizes: the item's values of the group's first fixed spectrum,
    // loaded with the slab tiles so that the product does not wait on them
    __shared__ cf sbuf[kFast ? 1 : 2 * NZ * W];
    __shared__ cf tw[NZ > 1 ? NZ : 1];
    __shared__ const cf* spec_of[GR];
    __shared__ int zr_of[GR][2];  // slab range [zlo, zhi] of each rotation of the group
    const int64_t G = int64_t(N) * N * NZ;
    if constexpr (NZ > 1) fill_twiddles<float, NZ>(tw);
    auto line_of = [](int r, int t, int cc) { return ((r & 1) * GR + (r >> 1) * 2 + t) * W + cc; };
    const int ngroups = (n_rot + GR - 1) / GR;
    const int items = (kFast ? pencil_jobs_grouped<N>() : pencil_jobs<N>()) * ngroups;
    const int npair = (n_rot + 1) / 2;
    constexpr int njobs = kFast ? pencil_jobs_grouped<N>() : pencil_jobs<N>();
    // The two-pass path gives each block a contiguous run of items, item =
    // job * ngroups + group, so consecutive items share the pencil job and
    // the spectrum values kept in registers; the generic path strides.
    const int per = (items + int(gridDim.x) - 1) / int(gridDim.x);
    const int ibeg = kFast ? int(blockIdx.x) * per : int(blockIdx.x);
    const int iend = kFast ? (ibeg + per < items ? ibeg + per : items) : items;
    const int istep = kFast ? 1 : int(gridDim.x);
    cf spre[kFast ? PencilSpec<N, GR>::kRows : 1][8];
    int prev_job = -1;
    const cf* prev_spec[GR];
#pragma unroll
    for (int k = 0; k < GR; ++k) prev_spec[k] = nullptr;
    if constexpr (kFast && PencilSpec<N, GR>::kPipe) {
        // raw columns of the block's first item, one chunk per wave (later
        // items' columns are loaded during the previous item's inverse passes)
        static_assert(PencilChunk<N, GR>::kChunks == kPencilBlock / 64, "one chunk per wave");
        if (ibeg < iend) {
            const int wave = uniform(int(threadIdx.x) >> 6), lane = int(threadIdx.x) & 63;
            cf v0[N / 8];
            pencil_load_chunk<N, GR>(slabs, rots, n_rot, pencil_job_grouped<N>(ibeg / ngroups), (ibeg % ngroups) * GR,
                                     wave, lane, v0);
            pencil_store_raw<N, GR>(buf, wave, lane, v0);
        }
    }
    for (int item = ibeg; item < iend; item += istep) {
        const int jobi = kFast ? item / ngroups : item % njobs;
        const PencilJob job = kFast ? pencil_job_grouped<N>(jobi) : pencil_job<N>(jobi);
        const int g0 = (kFast ? item % ngroups : item / njobs) * GR;  // first rotation of the group
        const int kyt[2] = {job.ky, (N - job.ky) % N};
        auto kx_of = [&](int t, int cc) { return t == 0 ? job.x0 + cc : (N - job.x0 - cc) % N; };
        __syncthreads();  // previous item done with buf / spec_of
        if (threadIdx.x < GR) {
            const int rot = g0 + threadIdx.x;
            spec_of[threadIdx.x] = rot < n_rot ? static_cast<const cf*>(jobs[rots[rot].job].spec) : nullptr;
            zr_of[threadIdx.x][0] = rot < n_rot ? (NZ > 1 ? int(rots[rot].zlo) : 0) : 1;
            zr_of[threadIdx.x][1] = rot < n_rot ? (NZ > 1 ? int(rots[rot].zhi) : 0) : 0;
        }
        __syncthreads();  // spec_of / zr_of visible
        if constexpr (kFast) {
            bool reload = jobi != prev_job;
#pragma unroll
            for (int k = 0; k < GR; ++k) {
                reload = reload || spec_of[k] != prev_spec[k];
                prev_spec[k] = spec_of[k];
            }
            prev_job = jobi;
            const int nitem = item + 1;
            const PencilNext nx{pencil_job_grouped<N>(nitem / ngroups), (nitem % ngroups) * GR, nitem < iend};
            pencil_item_fast<N, GR>(n_rot, rots, slabs, packed, buf, tw, spec_of, job, g0, nx, spre, reload);
            continue;
        }
        // load both tiles of every rotation of the group (zeros for missing
        // rotations) and the first rotation's spectrum values; all loads of a
        // thread are issued before its LDS writes
        {
            constexpr int TOT = GR * 2 * NZ * W;
            constexpr int PER = (TOT + kPencilBlock - 1) / kPencilBlock;
            constexpr int STOT = 2 * NZ * W;
            constexpr int SPER = (STOT + kPencilBlock - 1) / kPencilBlock;
            cf v[PER];
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int i = threadIdx.x + p * kPencilBlock;
                const int cc = i % W;
                const int kz = (i / W) % NZ;
                const int t = (i / (W * NZ)) % 2;
                const int r = i / (W * NZ * 2);
                const int rot = g0 + r;
                v[p] = mk(0.f, 0.f);
                const int zc = kz < NZ / 2 ? kz : kz - NZ;
                const bool reached = NZ == 1 || (zc >= zr_of[r][0] && zc <= zr_of[r][1]);
                if ((TOT % kPencilBlock == 0 || i < TOT) && rot < n_rot && reached)
                    v[p] = slabs[int64_t(rot) * G + (int64_t(kz) * N + kyt[t]) * N + kx_of(t, cc)];
            }
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int i = threadIdx.x + p * kPencilBlock;
                if (TOT % kPencilBlock == 0 || i < TOT) {
                    const int cc = i % W;
                    const int kz = (i / W) % NZ;
                    const int t = (i / (W * NZ)) % 2;
                    const int r = i / (W * NZ * 2);
                    buf[kz * NL + line_of(r, t, cc)] = v[p];
                }
            }
            const cf* sp0 = spec_of[0];  // the group's first rotation exists
            cf sv[SPER];
#pragma unroll
            for (int p = 0; p < SPER; ++p) {
                const int i = threadIdx.x + p * kPencilBlock;
                if (STOT % kPencilBlock == 0 || i < STOT) {
                    const int cc = i % W;
                    const int kz = (i / W) % NZ;
                    const int t = i / (W * NZ);
                    sv[p] = sp0[(int64_t(kz) * N + kyt[t]) * N + kx_of(t, cc)];
                }
            }
#pragma unroll
            for (int p = 0; p < SPER; ++p) {
                const int i = threadIdx.x + p * kPencilBlock;
                if (STOT % kPencilBlock == 0 || i < STOT) sbuf[i] = sv[p];
            }
        }
        __syncthreads();
        if constexpr (NZ == 96 && NL * 8 <= kPencilBlock)
            zfft_lines_r8<NZ, -1, NL, NL, kPencilBlock>(buf, tw);
        else if constexpr (NZ > 1)
            lds_fft_lines<float, NZ, -1, true, Plan>(buf, NL, 1, NL, tw);
        // product with each rotation's fixed spectrum (shared spectra hit in cache)
        for (int i = threadIdx.x; i < 2 * NZ * W; i += kPencilBlock) {
            const int cc = i % W;
            const int kz = (i / W) % NZ;
            const int t = i / (W * NZ);
            const int64_t off = (int64_t(kz) * N + kyt[t]) * N + kx_of(t, cc);
            const cf* prev = spec_of[0];
            cf sv = sbuf[i];
#pragma unroll
            for (int r = 0; r < GR; ++r) {
                const cf* sp = spec_of[r];
                if (sp == nullptr) continue;
                if (sp != prev) {
                    sv = sp[off];
                    prev = sp;
                }
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
        if constexpr (NZ == 96 && NL * 8 <= kPencilBlock)
            zfft_lines_r8<NZ, 1, NL, GR * W, kPencilBlock>(buf, tw);
        else if constexpr (NZ > 1)
            lds_fft_lines<float, NZ, 1, true, Plan>(buf, NL, 1, GR * W, tw);
        // write the folded pencils of each pair
        const int pair0 = g0 / 2;
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
}

// K2 for spectra that arrive already transformed along every axis and
// multiplied by the fixed spectrum (the nonequispaced route's modes, 3D,
// N = 64 and 128, in column tiles): fold rotation pairs and run the inverse z
// pass into the packed grids, so that K3 and K4 give the peaks as on the
// search path.  Same items and loads as the pencil kernel with groups of 2.
template <int N>
__global__ __launch_bounds__(kPencilBlock, 4) void pencil_modes_kernel(const FusedRot* __restrict__ rots, int n_rot,
                                                                    const cf* __restrict__ modes,
                                                                    cf* __restrict__ packed) {
    constexpr int GR = 2;
    constexpr int NL = 2 * pencil_width<N>() * GR;
    static_assert(SlabLayout<N>::kFast && PencilSpec<N, GR>::kPipe, "two-pass sizes");
    __shared__ cf buf[N * (NL + 8)];
    __shared__ cf tw[N];
    fill_twiddles<float, N>(tw);
    const int ngroups = (n_rot + GR - 1) / GR;
    const int items = pencil_jobs_grouped<N>() * ngroups;
    const int per = (items + int(gridDim.x) - 1) / int(gridDim.x);
    const int ibeg = int(blockIdx.x) * per, iend = ibeg + per < items ? ibeg + per : items;
    cf spre[PencilSpec<N, GR>::kRows][8];
    if (ibeg < iend) {
        const int wave = uniform(int(threadIdx.x) >> 6), lane = int(threadIdx.x) & 63;
        cf v0[N / 8];
        pencil_load_chunk<N, GR, true>(modes, rots, n_rot, pencil_job_grouped<N>(ibeg / ngroups),
                                       (ibeg % ngroups) * GR, wave, lane, v0);
        pencil_store_raw<N, GR, true>(buf, wave, lane, v0);
    }
    for (int item = ibeg; item < iend; ++item) {
        const PencilJob job = pencil_job_grouped<N>(item / ngroups);
        const int g0 = (item % ngroups) * GR;
        const int nitem = item + 1;
        const PencilNext nx{pencil_job_grouped<N>(nitem / ngroups), (nitem % ngroups) * GR, nitem < iend};
        __syncthreads();  // the previous item's loads are in buf
        pencil_item_fast<N, GR, true>(n_rot, rots, modes, packed, buf, tw, nullptr, job, g0, nx, spre, false);
    }
}

// descriptors of a batch of one pair's rotations for K3 / K4: rotation i
// writes its outputs at index i of the given arrays
__global__ void modes_desc_kernel(FusedRot* __restrict__ rots, int n, FusedJob* __restrict__ job, float* score,
                                  int32_t* t, float* nbhd, double* refined, int n_m) {
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i == 0) *job = FusedJob{nullptr, nullptr, nullptr, score, t, nbhd, refined, n_m, 0};
    if (i < n) {
        FusedRot r{};
        r.job = 0;
        r.local = i;
        r.zlo = -32768;
        r.zhi = 32767;
        rots[i] = r;
    }
}

// ------------------------------------------------------------------ K3
__device__ __forceinline__ bool better(float v, int i, float bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

// one step of the (max, lowest index) reduction with a DPP lane pattern
template <int CTRL>
__device__ __forceinline__ void argmax_dpp_step(float& v, int& i) {
    const float ov = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, 0xF, 0xF,
                                                                false));
    const int oi = __builtin_amdgcn_update_dpp(i, i, CTRL, 0xF, 0xF, false);
    if (better(ov, oi, v, i)) {
        v = ov;
        i = oi;
    }
}

// (max, lowest index) over the wave, in every lane.  Inside each row of 16
// lanes through DPP patterns (no LDS round trip): swap neighbours, swap
// pairs, mirror the half rows (quad 0 meets quad 1), mirror the row; then
// across rows with two shuffles.
__device__ __forceinline__ void wave_argmax(float& v, int& i) {
    argmax_dpp_step<0xB1>(v, i);   // quad_perm [1, 0, 3, 2]
    argmax_dpp_step<0x4E>(v, i);   // quad_perm [2, 3, 0, 1]
    argmax_dpp_step<0x141>(v, i);  // row_half_mirror
    argmax_dpp_step<0x140>(v, i);  // row_mirror
    for (int off = 16; off < warpSize; off <<= 1) {
        const float ov = __shfl_xor(v, off);
        const int oi = __shfl_xor(i, off);
        if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
}

__device__ __forceinline__ void take(float v, int i, float& bv, int& bi) {
    if (better(v, i, bv, bi)) {
        bv = v;
        bi = i;
    }
}

// Inverse 2D DFT of one folded slab (N = 8 R1, R1 = 8, 12 or 16) with the
// per-thread argmax of its real (rotation A) and imaginary (rotation B)
// parts.  Pass A (radix R1 along y) takes its inputs from registers loaded
// from global memory one item ahead; pass B (radix 8) runs in place; along x,
// 8 lanes own a row for both passes, and the outputs of the last pass go
// straight to the argmax.  `pre` holds this item's pass-A inputs on entry
// and the next item's (loaded from `next`, if not null) on return: the loads
// are in flight during the x passes.
template <int N>
__device__ __forceinline__ void islab_fft_argmax_fast(cf* pre, const cf* __restrict__ next, cf* __restrict__ slab,
                                                      const cf* __restrict__ tw, int zoff, float& va, int& ia,
                                                      float& vb, int& ib, bool grouped) {
    constexpr int R1 = N / 8;
    constexpr int NB = N / 8;
    // row entry e at e + e / 16: the radix-16 pass along x writes 16
    // consecutive entries per lane, which without the gap would put the 8
    // lanes of a row on the same banks
    constexpr int RS = N + N / 16 + 4;  // padded row stride (complex entries)
    auto px = [](int e) { return e + (e >> 4); };
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int x = t % N, jb = t / N;
    const bool on = jb < 8;
    if (on) {
        dftR<float, 1, R1>(pre);
#pragma unroll
        for (int r = 0; r < R1; ++r) slab[(jb * R1 + r) * RS + px(x)] = pre[r];
    }
    __syncthreads();
    if (on) {
#pragma unroll
        for (int m = 0; m < (NB + 7) / 8; ++m) {
            const int jj = jb + 8 * m;
            if (NB % 8 != 0 && jj >= NB) break;  // R1 = 12: lanes 0-3 take a second butterfly
            cf u[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) u[r] = slab[(jj + NB * r) * RS + px(x)];
#pragma unroll
            for (int r = 1; r < 8; ++r) u[r] = u[r] * conj(tw[r * jj]);
            dft8<float, 1>(u);
#pragma unroll
            for (int r = 0; r < 8; ++r) slab[(jj + NB * r) * RS + px(x)] = u[r];
        }
        if (next) {
            const int px = grouped ? col_pos<N>(x) : x;
#pragma unroll
            for (int r = 0; r < R1; ++r) pre[r] = next[(jb + 8 * r) * N + px];
        }
    }
    __syncthreads();
    const int y = t / 8, j = t % 8;
    if (y < N) {
        cf v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = slab[y * RS + px(j + 8 * r)];
        compiler_fence();
        dftR<float, 1, R1>(v);
#pragma unroll
        for (int r = 0; r < R1; ++r) slab[y * RS + px(j * R1 + r)] = v[r];
        compiler_fence();
        constexpr int MB = (NB + 7) / 8;  // butterflies per lane (lanes 0-3 of N = 96 take 2, 4-7 take 1)
        const bool two = NB % 8 == 0 || j + 8 * (MB - 1) < NB;
        cf u[MB][8];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int jj = j + 8 * m;
            if (NB % 8 != 0 && m == MB - 1 && !two) break;
#pragma unroll
            for (int r = 0; r < 8; ++r) u[m][r] = slab[y * RS + px(jj + NB * r)];
#pragma unroll
            for (int r = 1; r < 8; ++r) u[m][r] = u[m][r] * conj(tw[r * jj]);
            dft8<float, 1>(u[m]);
        }
        // visit the outputs in increasing index (x = j + 8 m + NB r): a
        // strict comparison then keeps the lowest index among equal values;
        // the slot (x - j) / 8 when NB is a multiple of 8, else x - j, is
        // turned into the flat index once
        constexpr int SU = NB % 8 == 0 ? 8 : 1;  // index units per slot
        int sa = -1, sb = -1;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                if (NB % 8 != 0 && m == MB - 1 && !two) continue;
                const int slot = (8 * m + NB * r) / SU;
                if (u[m][r].re > va) { va = u[m][r].re; sa = slot; }
                if (u[m][r].im > vb) { vb = u[m][r].im; sb = slot; }
            }
        }
        const int row = zoff + y * N + j;
        if (sa >= 0) ia = row + SU * sa;
        if (sb >= 0) ib = row + SU * sb;
    }
}

// Work item = (z-slab, rotation pair), z fastest.
template <int N, int P>
__global__ __launch_bounds__(slab_block(N)) void islab_peak_kernel(const cf* __restrict__ packed, int nz, int n_rot,
                                                                    float* __restrict__ pval, int* __restrict__ pidx) {
    constexpr int B = slab_block(N), NW = islab_waves(N);
    using Plan = typename FusedRadix<N, P>::type;
    // register-resident transform: the fast sizes (pair-grouped columns in
    // 3D) and N = 96 (radix 12 x 8, row-major slabs)
    constexpr bool kFast = SlabLayout<N>::kRowFft;
    constexpr int TPL = slab_tpl<N>(), RS = slab_pitch<N>();  // generic sizes
    __shared__ cf slab[kFast ? N * (N + N / 16 + 4) : N * RS];
    __shared__ cf tw[N];
    fill_twiddles<float, N>(tw);
    const int npair = (n_rot + 1) / 2;
    const int items = nz * npair;
    const bool grouped = nz == N && SlabLayout<N>::kFast;
    auto src_of = [&](int item) { return packed + (int64_t(item / nz) * nz + item % nz) * N * N; };
    cf pre[kFast ? N / 8 : 1];
    if constexpr (kFast) {
        const int x = threadIdx.x % N, jb = threadIdx.x / N;
        if (int(blockIdx.x) < items && jb < 8) {
            const cf* src = src_of(blockIdx.x);
            const int px = grouped ? col_pos<N>(x) : x;
#pragma unroll
            for (int r = 0; r < N / 8; ++r) pre[r] = src[(jb + 8 * r) * N + px];
        }
    }
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int z = item % nz, pair = item / nz;
        const cf* src = src_of(item);
        float va = -INFINITY, vb = -INFINITY;
        int ia = 0x7fffffff, ib = 0x7fffffff;
        const int zoff = z * N * N;
        __syncthreads();
        if constexpr (kFast) {
            const int nx = item + int(gridDim.x);
            islab_fft_argmax_fast<N>(pre, nx < items ? src_of(nx) : nullptr, slab, tw, zoff, va, ia, vb, ib,
                                     grouped);
        } else {
            stage_rows_to_lds<N, RS, B>(reinterpret_cast<float4*>(slab), reinterpret_cast<const float4*>(src));
            __syncthreads();
            lds_fft_lines<float, N, 1, true, Plan, TPL>(slab, RS, 1, N, tw);   // along y
            lds_fft_lines<float, N, 1, false, Plan, TPL>(slab, 1, RS, N, tw);  // along x
            for (int i = threadIdx.x; i < N * N; i += B) {
                const cf v = slab[(i / N) * RS + i % N];
                take(v.re, zoff + i, va, ia);
                take(v.im, zoff + i, vb, ib);
            }
        }
        // one partial per wave, reduced by the finish kernel: no barrier and
        // no serial tail between items
        wave_argmax(va, ia);
        wave_argmax(vb, ib);
        const int lane = threadIdx.x % warpSize, wid = threadIdx.x / warpSize;
        if (lane == 0) {
            const int64_t at = (int64_t(2 * pair) * nz + z) * NW + wid;
            pval[at] = va;
            pidx[at] = ia;
            if (2 * pair + 1 < n_rot) {
                pval[at + int64_t(nz) * NW] = vb;
                pidx[at + int64_t(nz) * NW] = ib;
            }
        }
    }
}

// ------------------------------------------------------------------ K4
// (dz, rotation): peak from the per-wave slab partials, then the 9 scores of slab
// t_z + dz around (t_x, t_y) by a separable inverse DFT of the folded slab:
//   h_j(ky)  = sum_kx P(kx, ky) e^{2 pi i kx x_j / N},  x_j in t_x + {-1, 0, 1}
//   g(x_j, y_i) = sum_ky h_j(ky) e^{2 pi i ky y_i / N}
// Re g belongs to the even rotation of the pair, Im g to the odd one.
template <int N>
__global__ __launch_bounds__(kFinishBlock) void finish_slab_kernel(const cf* __restrict__ packed, int nz,
                                                                   const float* __restrict__ pval,
                                                                   const int* __restrict__ pidx,
                                                                   double* __restrict__ nbbuf,
                                                                   const FusedRot* __restrict__ rots,
                                                                   const FusedJob* __restrict__ jobs) {
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
    constexpr int NW = islab_waves(N);
    {
        // every partial of the thread loaded before the first comparison (the
        // (value, lowest index) order is total, so the visiting order does
        // not matter); nz is N or 1
        constexpr int PB = (N * NW + kFinishBlock - 1) / kFinishBlock;
        const float* pv = pval + int64_t(rot) * nz * NW;
        const int* pi = pidx + int64_t(rot) * nz * NW;
        float vv[PB];
        int ii[PB];
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int i = int(threadIdx.x) + p * kFinishBlock;
            vv[p] = -INFINITY;
            ii[p] = 0x7fffffff;
            if (i < nz * NW) {
                vv[p] = pv[i];
                ii[p] = pi[i];
            }
        }
#pragma unroll
        for (int p = 0; p < PB; ++p)
            if (better(vv[p], ii[p], bv, bi)) { bv = vv[p]; bi = ii[p]; }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kFinishBlock / 2; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off && better(sv[threadIdx.x + off], si[threadIdx.x + off], sv[threadIdx.x], si[threadIdx.x])) {
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
    // inner sums along x: two threads per row ky, each half of the row's
    // stored positions
    const bool grouped = nz == N && (N == 64 || N == 128);
    // (the loads of HB positions are issued together: one at a time, each
    // waited on before the next, the loop ran at cache latency)
    constexpr int HB = N / 2 >= 16 ? 16 : N / 2;
    static_assert((N / 2) % HB == 0, "whole batches of positions");
    for (int w = threadIdx.x; w < 2 * N; w += kFinishBlock) {
        const int ky = w >> 1, half = w & 1;
        double ar[3] = {0, 0, 0}, ai[3] = {0, 0, 0};
        for (int p0 = half * (N / 2); p0 < (half + 1) * (N / 2); p0 += HB) {
            cf vb[HB];
#pragma unroll
            for (int q = 0; q < HB; ++q) vb[q] = sl[ky * N + p0 + q];
#pragma unroll
            for (int q = 0; q < HB; ++q) {
                const int px = p0 + q;
                const int kx = grouped ? col_kx<N>(px) : px;
                const double vr = vb[q].re, vi = vb[q].im;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int m = (kx * xs[j]) % N;
                    ar[j] += vr * twr[m] - vi * twi[m];
                    ai[j] += vr * twi[m] + vi * twr[m];
                }
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
        const FusedRot fr = rots[rot];
        const FusedJob jb = jobs[fr.job];
        jb.score[fr.local] = bv;
        jb.t[3 * fr.local] = tx;
        jb.t[3 * fr.local + 1] = ty;
        jb.t[3 * fr.local + 2] = tz;
    }
}

// per rotation: neighbourhood out, per-axis parabola vertex in FP64
__global__ void finish_rot_kernel(const double* __restrict__ nbbuf, const FusedRot* __restrict__ rots,
                                  const FusedJob* __restrict__ jobs, int n_rot) {
    const int rot = blockIdx.x * blockDim.x + threadIdx.x;
    if (rot >= n_rot) return;
    const FusedRot fr = rots[rot];
    const FusedJob jb = jobs[fr.job];
    const int loc = fr.local;
    const double* nb = nbbuf + 27 * int64_t(rot);
    if (jb.nbhd)
        for (int a = 0; a < 27; ++a) jb.nbhd[27 * int64_t(loc) + a] = float(nb[a]);
    if (jb.refined) {
        const int32_t* tout = jb.t;
        double* refined = jb.refined;
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
            refined[3 * loc + a] = double(tout[3 * loc + a]) + d;
        }
    }
}

// launch, recording the kernel's own start / stop timestamps when timed
template <typename F, typename... Args>
void launch_k(KernelTimer* kt, const char* name, F kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    if (kt) {
        hipEvent_t a = nullptr, b = nullptr;
        kt->events(name, &a, &b);
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    }
}

struct FusedLayout {
    cf* slabs;
    cf* packed;
    float* pval;
    int* pidx;
    double* nbbuf;
    size_t total;
};

FusedLayout fused_layout(const FusedPlan& fp, void* ws) {
    const int nz = fp.planar ? 1 : fp.N;
    const int64_t G = int64_t(fp.N) * fp.N * nz;
    char* base = static_cast<char*>(ws);
    FusedLayout L{};
    size_t off = 0;
    L.slabs = reinterpret_cast<cf*>(base + off);
    off += align256(sizeof(cf) * G * fp.batch);
    L.packed = reinterpret_cast<cf*>(base + off);
    off += align256(sizeof(cf) * G * ((fp.batch + 1) / 2));
    L.pval = reinterpret_cast<float*>(base + off);
    off += align256(sizeof(float) * nz * islab_waves(fp.N) * fp.batch);
    L.pidx = reinterpret_cast<int*>(base + off);
    off += align256(sizeof(int) * nz * islab_waves(fp.N) * fp.batch);
    L.nbbuf = reinterpret_cast<double*>(base + off);
    off += align256(sizeof(double) * 27 * fp.batch);
    L.total = off;
    return L;
}

unsigned persistent_grid(int items, int cap) {
    if (cap <= 0 || items <= cap) return unsigned(items > 0 ? items : 1);
    return unsigned(cap);
}

// Slab kernel blocks resident per compute unit (N = 64: two spread blocks
// and four inverse slab blocks of 512 threads), from the occupancy query, so
// that a persistent grid never holds blocks that wait for others to finish.
template <int N, int P>
int spread_blocks_per_cu() {
    static const int n = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, spread_slab_kernel<N, P>, slab_block(N), 0) != hipSuccess)
            b = 1;
        return b < 1 ? 1 : b;
    }();
    return n;
}

template <int N, int P>
int islab_blocks_per_cu() {
    static const int n = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, islab_peak_kernel<N, P>, slab_block(N), 0) != hipSuccess)
            b = 1;
        return b < 1 ? 1 : b;
    }();
    return n;
}

template <int N, int P>
hipError_t fused_impl(const FusedPlan& fp, const FusedRot* rots, int n_rot, const FusedJob* jobs, void* ws,
                      hipStream_t s, KernelTimer* kt) {
    const int nz = fp.planar ? 1 : N;
    const int npair = (n_rot + 1) / 2;
    const FusedLayout L = fused_layout(fp, ws);
    launch_k(kt, "spread_slab", spread_slab_kernel<N, P>,
             dim3(persistent_grid(nz * n_rot, fp.max_wgs * spread_blocks_per_cu<N, P>())), dim3(slab_block(N)), s,
             rots, jobs, n_rot, fp.planar ? 1 : 0, L.slabs);
    const int gr = fp.pencil_group;
    const int items2 = (fused_pair_grouped(N, fp.planar) ? pencil_jobs_grouped<N>() : pencil_jobs<N>()) *
                       ((n_rot + gr - 1) / gr);
    const dim3 g2{persistent_grid(items2, fp.max_wgs * (gr == 2 ? 2 : 1)), 1u, 1u};
    const dim3 b2{unsigned(kPencilBlock), 1u, 1u};
    if (fp.planar) {
        if (gr == 4)
            launch_k(kt, "pencil", pencil_kernel<N, 1, 4, P>, g2, b2, s, rots, jobs, n_rot, L.slabs, L.packed);
        else
            launch_k(kt, "pencil", pencil_kernel<N, 1, 2, P>, g2, b2, s, rots, jobs, n_rot, L.slabs, L.packed);
    } else {
        if (gr == 4)
            launch_k(kt, "pencil", pencil_kernel<N, N, 4, P>, g2, b2, s, rots, jobs, n_rot, L.slabs, L.packed);
        else
            launch_k(kt, "pencil", pencil_kernel<N, N, 2, P>, g2, b2, s, rots, jobs, n_rot, L.slabs, L.packed);
    }
    launch_k(kt, "islab_peak", islab_peak_kernel<N, P>,
             dim3(persistent_grid(nz * npair, fp.max_wgs * islab_blocks_per_cu<N, P>())), dim3(slab_block(N)), s,
             L.packed, nz, n_rot, L.pval, L.pidx);
    const dim3 g4{unsigned(fp.planar ? 1 : 3), unsigned(n_rot), 1u};
    launch_k(kt, "finish", finish_slab_kernel<N>, g4, dim3(kFinishBlock), s, L.packed, nz, L.pval, L.pidx, L.nbbuf,
             rots, jobs);
    launch_k(kt, "finish_rot", finish_rot_kernel, dim3(unsigned((n_rot + 63) / 64)), dim3(64), s, L.nbbuf, rots, jobs,
             n_rot);
    return hipGetLastError();
}

template <int N>
hipError_t fused_dispatch(const FusedPlan& fp, const FusedRot* rots, int n_rot, const FusedJob* jobs, void* ws,
                          hipStream_t s, KernelTimer* kt) {
    switch (fp.radix) {
        case 0: return fused_impl<N, 0>(fp, rots, n_rot, jobs, ws, s, kt);
        case 1: return fused_impl<N, 1>(fp, rots, n_rot, jobs, ws, s, kt);
        case 2: return fused_impl<N, 2>(fp, rots, n_rot, jobs, ws, s, kt);
        default: return hipErrorInvalidValue;
    }
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ void fill_random_kernel(cf* __restrict__ p, int64_t n, uint32_t seed, float amp) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) {
        const uint32_t a = hash32(uint32_t(i) * 2u + seed * 0x9e3779b9U);
        const uint32_t b = hash32(uint32_t(i) * 2u + 1u + seed * 0x9e3779b9U);
        p[i] = mk(amp * (float(a) * 2.3283064e-10f - 0.5f), amp * (float(b) * 2.3283064e-10f - 0.5f));
    }
}

struct ModesLayout {
    cf* packed;
    float* pval;
    int* pidx;
    double* nbbuf;
    FusedRot* rots;
    FusedJob* job;
    size_t total;
};

ModesLayout modes_layout(int N, int nb, void* ws) {
    const int64_t G = int64_t(N) * N * N;
    char* base = static_cast<char*>(ws);
    ModesLayout L{};
    size_t off = 0;
    L.packed = reinterpret_cast<cf*>(base + off);
    off += align256(sizeof(cf) * G * ((nb + 1) / 2));
    L.pval = reinterpret_cast<float*>(base + off);
    off += align256(sizeof(float) * N * islab_waves(N) * size_t(nb));
    L.pidx = reinterpret_cast<int*>(base + off);
    off += align256(sizeof(int) * N * islab_waves(N) * size_t(nb));
    L.nbbuf = reinterpret_cast<double*>(base + off);
    off += align256(sizeof(double) * 27 * size_t(nb));
    L.rots = reinterpret_cast<FusedRot*>(base + off);
    off += align256(sizeof(FusedRot) * size_t(nb));
    L.job = reinterpret_cast<FusedJob*>(base + off);
    off += align256(sizeof(FusedJob));
    L.total = off;
    return L;
}

template <int N>
hipError_t modes_peaks_impl(const cf* modes, int nb, int n_m, float* score, int32_t* t, float* nbhd, double* refined,
                            int num_cu, void* ws, hipStream_t s) {
    const ModesLayout L = modes_layout(N, nb, ws);
    hipLaunchKernelGGL(modes_desc_kernel, dim3(unsigned((nb + 255) / 256)), dim3(256), 0, s, L.rots, nb, L.job,
                       score, t, nbhd, refined, n_m);
    const int items2 = pencil_jobs_grouped<N>() * ((nb + 1) / 2);
    hipLaunchKernelGGL(pencil_modes_kernel<N>, dim3(persistent_grid(items2, 2 * num_cu)), dim3(kPencilBlock), 0, s,
                       L.rots, nb, modes, L.packed);
    hipLaunchKernelGGL((islab_peak_kernel<N, 0>),
                       dim3(persistent_grid(N * ((nb + 1) / 2), num_cu * islab_blocks_per_cu<N, 0>())),
                       dim3(slab_block(N)), 0, s, L.packed, N, nb, L.pval, L.pidx);
    hipLaunchKernelGGL(finish_slab_kernel<N>, dim3(3u, unsigned(nb)), dim3(kFinishBlock), 0, s, L.packed, N, L.pval,
                       L.pidx, L.nbbuf, L.rots, L.job);
    hipLaunchKernelGGL(finish_rot_kernel, dim3(unsigned((nb + 63) / 64)), dim3(64), 0, s, L.nbbuf, L.rots, L.job, nb);
    return hipGetLastError();
}

}  // namespace

size_t fused_workspace_bytes(const FusedPlan& fp) { return fused_layout(fp, nullptr).total; }

namespace {
template <int N>
void query_slab_kernels() {
    (void)spread_blocks_per_cu<N, 0>();
    (void)spread_blocks_per_cu<N, 1>();
    (void)spread_blocks_per_cu<N, 2>();
    (void)islab_blocks_per_cu<N, 0>();
    (void)islab_blocks_per_cu<N, 1>();
    (void)islab_blocks_per_cu<N, 2>();
}
}  // namespace

void fused_query_occupancy() {
    query_slab_kernels<8>();
    query_slab_kernels<16>();
    query_slab_kernels<32>();
    query_slab_kernels<64>();
    query_slab_kernels<96>();
    query_slab_kernels<128>();
}

bool modes_peaks_supported(int N, bool planar) { return fused_pair_grouped(N, planar); }

size_t modes_peaks_workspace_bytes(int N, int nb) { return modes_layout(N, nb, nullptr).total; }

hipError_t launch_modes_peaks(int N, const void* modes, int nb, int n_m, float* score, int32_t* t, float* nbhd,
                              double* refined, int num_cu, void* ws, hipStream_t s) {
    const cf* m = static_cast<const cf*>(modes);
    switch (N) {
        case 64: return modes_peaks_impl<64>(m, nb, n_m, score, t, nbhd, refined, num_cu, ws, s);
        case 128: return modes_peaks_impl<128>(m, nb, n_m, score, t, nbhd, refined, num_cu, ws, s);
        default: return hipErrorInvalidValue;
    }
}

size_t fused_prep_scratch_bytes(int n_jobs) { return align256(sizeof(float) * kPrepBlocks * size_t(n_jobs)); }

// The copy also multiplies S(k) by (-1)^(kx + ky) / 2: the slabs of these
// sizes are spread at positions shifted by N / 2 in x and y, so their
// transforms carry the sign, and (-1)^(kx + ky) is the same at k and -k, so
// the product Y(k) S(k) that the pencil pass folds is unchanged; the 1/2 is
// the fold's own factor in H(k) = (Y(k) + conj(Y(-k))) / 2 (an exact power of
// two, so the folded values are the same).
template <int N>
__global__ void spec_pair_group_kernel(const cf* __restrict__ in, cf* __restrict__ out) {
    const int64_t rows = int64_t(N) * N;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < rows * N; i += int64_t(gridDim.x) * blockDim.x) {
        const int p = int(i % N);
        const int kx = col_kx<N>(p), ky = int((i / N) % N), kz = int(i / rows);
        const cf v = in[i - p + kx];
        const float h = ((kx + ky) & 1) ? -0.5f : 0.5f;
        out[tile_index<N>(kz, ky, p)] = mk(h * v.re, h * v.im);
    }
}

hipError_t launch_spec_pair_group(const void* spec, void* out, int N, hipStream_t s) {
    const cf* in = static_cast<const cf*>(spec);
    cf* o = static_cast<cf*>(out);
    if (N == 128)
        hipLaunchKernelGGL(spec_pair_group_kernel<128>, dim3(2048), dim3(256), 0, s, in, o);
    else if (N == 64)
        hipLaunchKernelGGL(spec_pair_group_kernel<64>, dim3(1024), dim3(256), 0, s, in, o);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_rot_desc(const RotInput* in, int64_t n, FusedRot* out, hipStream_t s) {
    hipLaunchKernelGGL(rot_desc_kernel, dim3(unsigned((n + 63) / 64)), dim3(64), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_fused_prep(const FusedJob* jobs, int n_jobs, void* scratch, hipStream_t s) {
    float* part = static_cast<float*>(scratch);
    const dim3 g1{unsigned(kPrepBlocks), unsigned(n_jobs), 1u};
    hipLaunchKernelGGL(cmax_partial_kernel, g1, dim3(256), 0, s, jobs, part);
    hipLaunchKernelGGL(cmax_final_kernel, dim3(unsigned(n_jobs)), dim3(64), 0, s, jobs, part, kPrepBlocks);
    return hipGetLastError();
}

hipError_t launch_fused_batch(const FusedPlan& fp, const FusedRot* rots, int n_rot, const FusedJob* jobs, void* ws,
                              hipStream_t s, KernelTimer* kt) {
    switch (fp.N) {
        case 8: return fused_dispatch<8>(fp, rots, n_rot, jobs, ws, s, kt);
        case 16: return fused_dispatch<16>(fp, rots, n_rot, jobs, ws, s, kt);
        case 32: return fused_dispatch<32>(fp, rots, n_rot, jobs, ws, s, kt);
        case 64: return fused_dispatch<64>(fp, rots, n_rot, jobs, ws, s, kt);
        case 96: return fused_dispatch<96>(fp, rots, n_rot, jobs, ws, s, kt);
        case 128: return fused_dispatch<128>(fp, rots, n_rot, jobs, ws, s, kt);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fill_random(void* data, int64_t count, uint32_t seed, float amp, hipStream_t s) {
    hipLaunchKernelGGL(fill_random_kernel, dim3(1024), dim3(256), 0, s, static_cast<cf*>(data), count, seed, amp);
    return hipGetLastError();
}

}  // namespace sdf
