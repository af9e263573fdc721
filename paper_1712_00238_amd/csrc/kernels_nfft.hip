// Nonequispaced route of the search (Implementation section): octree-
// adaptive samples of the moving affinity, and per rotation the type-1
// nonequispaced transform of the rotated samples by "exponential of
// semicircle" spreading on the 2x oversampled grid, FFT, crop and
// deconvolution (Barnett, Magland and af Klinteberg, 2019), followed by the
// spectral product with the fixed part.
//
// Octree reading: cells of 2^l nodes per side (l <= max_level <= 3, aligned
// to multiples of 2^l) whose coefficient spread (max - min of Re and of Im)
// is below tol * A, A = max_k max(|Re c_k|, |Im c_k|), become one leaf at
// the cell centre carrying the sum of the cell's coefficients; each node
// goes to the highest such cell above it, or stays a leaf of its own.
// Leaves whose nodes are all zero are dropped.  Leaves are emitted per
// 8^3 (planar 8^2) block in flat block order, Morton order within a block.
#include <hip/hip_runtime.h>


#include <type_traits>

#include "common.hpp"
#include "fft.hpp"
#include "fft256.hpp"
#include "launch.hpp"

namespace sdf {
namespace {

template <typename T>
struct UBits;
template <>
struct UBits<float> {
    using U = unsigned int;
};
template <>
struct UBits<double> {
    using U = unsigned long long;
};

__device__ __forceinline__ float from_bits(unsigned int u) { return __uint_as_float(u); }
__device__ __forceinline__ double from_bits(unsigned long long u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ unsigned int to_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ unsigned long long to_bits(double v) {
    return (unsigned long long)__double_as_longlong(v);
}

__device__ __forceinline__ float dmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double dmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float dmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double dmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float dabs(float a) { return fabsf(a); }
__device__ __forceinline__ double dabs(double a) { return fabs(a); }
__device__ __forceinline__ float dceil(float a) { return ceilf(a); }
__device__ __forceinline__ double dceil(double a) { return ceil(a); }
__device__ __forceinline__ float dexp(float a) { return expf(a); }
__device__ __forceinline__ double dexp(double a) { return exp(a); }
__device__ __forceinline__ float dsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }

// ------------------------------------------------------------------ octree
template <typename U>
__global__ void clear_bits_kernel(U* p) {
    if (threadIdx.x == 0) p[0] = U(0);
}

// A as the bit pattern of a non-negative value: integer max orders such
// patterns like the values, so the result is exact and order-independent.
template <typename T>
__global__ __launch_bounds__(256) void absmax_kernel(const cplx<T>* __restrict__ c, int64_t n,
                                                     typename UBits<T>::U* __restrict__ out) {
    T m = T(0);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const cplx<T> v = c[i];
        m = dmax(m, dmax(dabs(v.re), dabs(v.im)));
    }
    __shared__ T wmax[4];
    for (int off = 32; off > 0; off >>= 1) m = dmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = dmax(dmax(wmax[0], wmax[1]), dmax(wmax[2], wmax[3]));
        if (m > T(0)) atomicMax(out, to_bits(m));  // one atomic per block
    }
}

constexpr int kOctBlock = 512;

// One block per 8^DIM node block, thread t = Morton index (x bit lowest).
// Level-l cells are runs of 2^(DIM l) consecutive threads, reduced with
// butterflies inside a wave and through LDS across the 8 waves (3D, l = 3).
// EMIT = false counts the block's leaves; EMIT = true writes them at
// offsets[block] + (leaves of lower threads).
template <typename T, int DIM, bool EMIT>
__global__ __launch_bounds__(kOctBlock) void octree_kernel(const cplx<T>* __restrict__ c, int nm,
                                                           const typename UBits<T>::U* __restrict__ amax, T tol,
                                                           int max_level, int* __restrict__ counts,
                                                           const int* __restrict__ offsets, T* __restrict__ pos,
                                                           cplx<T>* __restrict__ out_c, int* __restrict__ out_level) {
    constexpr int NT = DIM == 3 ? 512 : 64;
    constexpr int NW = NT / 64;
    __shared__ T s_mnr[NW], s_mxr[NW], s_mni[NW], s_mxi[NW];
    __shared__ double s_sr[NW], s_si[NW];
    __shared__ int s_nz[NW], s_cnt[NW];
    const int t = int(threadIdx.x), lane = t & 63, wq = t >> 6;
    int lx = 0, ly = 0, lz = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        lx |= ((t >> (DIM * b)) & 1) << b;
        ly |= ((t >> (DIM * b + 1)) & 1) << b;
        if (DIM == 3) lz |= ((t >> (DIM * b + 2)) & 1) << b;
    }
    const unsigned nb = unsigned(nm >> 3);
    const int bx = int(blockIdx.x % nb), by = int((blockIdx.x / nb) % nb);
    const int bz = DIM == 3 ? int(blockIdx.x / (nb * nb)) : 0;
    const int i = bx * 8 + lx, j = by * 8 + ly, k = bz * 8 + lz;
    const cplx<T> v = c[(int64_t(k) * nm + j) * nm + i];
    const T tau = tol * from_bits(amax[0]);

    T mnr = v.re, mxr = v.re, mni = v.im, mxi = v.im;
    double sr = double(v.re), si = double(v.im);
    int nz = (v.re != T(0) || v.im != T(0)) ? 1 : 0;
    // the leaf this node belongs to: its level and the cell's sums
    int lv = 0;
    double csr = sr, csi = si;
    int cnz = nz;
#pragma unroll
    for (int l = 1; l <= 3; ++l) {
#pragma unroll
        for (int b = DIM * (l - 1); b < DIM * l; ++b) {
            if (b < 6) {
                const int off = 1 << b;
                mnr = dmin(mnr, __shfl_xor(mnr, off));
                mxr = dmax(mxr, __shfl_xor(mxr, off));
                mni = dmin(mni, __shfl_xor(mni, off));
                mxi = dmax(mxi, __shfl_xor(mxi, off));
                sr += __shfl_xor(sr, off);
                si += __shfl_xor(si, off);
                nz |= __shfl_xor(nz, off);
            }
        }
        if (DIM * l > 6) {
            // every lane holds its wave's values; combine the waves in order
            if (lane == 0) {
                s_mnr[wq] = mnr;
                s_mxr[wq] = mxr;
                s_mni[wq] = mni;
                s_mxi[wq] = mxi;
                s_sr[wq] = sr;
                s_si[wq] = si;
                s_nz[wq] = nz;
            }
            __syncthreads();
            mnr = s_mnr[0];
            mxr = s_mxr[0];
            mni = s_mni[0];
            mxi = s_mxi[0];
            sr = s_sr[0];
            si = s_si[0];
            nz = s_nz[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                mnr = dmin(mnr, s_mnr[w]);
                mxr = dmax(mxr, s_mxr[w]);
                mni = dmin(mni, s_mni[w]);
                mxi = dmax(mxi, s_mxi[w]);
                sr += s_sr[w];
                si += s_si[w];
                nz |= s_nz[w];
            }
        }
        // spreads only grow with the cell, so the flat levels <= max_level
        // run from 1 up to some level; the last one is the leaf
        if (l <= max_level && (mxr - mnr < tau) && (mxi - mni < tau)) {
            lv = l;
            csr = sr;
            csi = si;
            cnz = nz;
        }
    }
    const bool keep = ((t & ((1 << (DIM * lv)) - 1)) == 0) && cnz != 0;
    const unsigned long long bal = __ballot(keep);
    if (lane == 0) s_cnt[wq] = __popcll(bal);
    __syncthreads();
    if (!EMIT) {
        if (t == 0) {
            int tot = 0;
            for (int w = 0; w < NW; ++w) tot += s_cnt[w];
            counts[blockIdx.x] = tot;
        }
        return;
    }
    if (!keep) return;
    int at = offsets[blockIdx.x];
    for (int w = 0; w < wq; ++w) at += s_cnt[w];
    at += __popcll(bal & ((1ull << lane) - 1ull));
    const T hs = T(0.5) * T((1 << lv) - 1), hm = T(0.5) * T(nm);
    pos[3 * int64_t(at)] = T(i) + hs - hm;
    pos[3 * int64_t(at) + 1] = T(j) + hs - hm;
    pos[3 * int64_t(at) + 2] = DIM == 3 ? T(k) + hs - hm : T(0);
    out_c[at] = mk(T(csr), T(csi));
    if (out_level) out_level[at] = lv;
}

__global__ void octree_total_kernel(const int* __restrict__ counts, const int* __restrict__ offsets, int nblk,
                                    int64_t* __restrict__ out) {
    if (threadIdx.x == 0) out[0] = int64_t(offsets[nblk - 1]) + counts[nblk - 1];
}

// ------------------------------------------------------------------ type-1 transform
constexpr double kEsBetaPerWidth = 2.30;  // beta = 2.30 w at oversampling 2
constexpr int kEsQuad = 4096;

// inv[j] = 1 / phihat(kappa_j), kappa_j = j (j < N/2) or j - N, with
// phihat(kappa) = int phi(2x/w) cos(2 pi kappa x / (2N)) dx over |x| <= w/2.
// With 2x/w = sin(theta) the integrand exp(beta (cos theta - 1))
// cos(pi kappa w sin(theta) / (2N)) (w/2) cos(theta) is smooth on
// [-pi/2, pi/2] (the square-root edge of phi is gone), so composite Simpson
// in FP64 converges fast even for narrow kernels, whose edge value e^-beta
// is not small.
template <typename T>
__global__ __launch_bounds__(256) void es_deconv_kernel(int N, int w, T* __restrict__ inv) {
    __shared__ double red[4];
    const int jj = int(blockIdx.x);
    const double kap = jj < N / 2 ? double(jj) : double(jj - N);
    const double beta = kEsBetaPerWidth * w, half = 0.5 * w, h = M_PI / kEsQuad;
    double acc = 0.0;
    // interior Simpson nodes q = 1 .. kEsQuad - 1; the end points contribute cos(+-pi/2) = 0
    for (int q = 1 + int(threadIdx.x); q < kEsQuad; q += 256) {
        const double th = -0.5 * M_PI + q * h;
        double st, ct;
        sincos(th, &st, &ct);
        const double g = exp(beta * (ct - 1.0)) * cospi(kap * half * st / double(N)) * half * ct;
        acc += (q & 1 ? 4.0 : 2.0) * g;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) inv[jj] = T(1.0 / ((red[0] + red[1] + red[2] + red[3]) * h / 3.0));
}

// ------------------------------------------------------------------ tiled spreading
// The oversampled grid is cut into tiles: general tiles of at most 4096 nodes
// (3D 32 x 16 x 8, planar 64 x 64, clipped to the grid; FP64 and planar) or,
// for FP32 3D, line tiles of whole x lines (below).  Per rotation each sample
// is binned by the tile that holds its first kernel node l0 = ceil(v - w/2),
// v being the reflected rotated position on the 2x grid wrapped to [0, 2N).
// A sample's w nodes per axis then lie in that tile or the ones just above,
// so a tile gathers the samples of its own bin and of the bins just below it
// (one per axis where w is at most the tile side), accumulates its nodes in
// LDS and stores each node once (no zero pass, no global atomics).
struct TileShape {
    int tx, ty, tz;     // tile sides in nodes
    int ntx, nty, ntz;  // tiles per axis
    int py, pz;         // LDS pitches of a row and a plane (padded against bank conflicts)
};
constexpr int kTileLds = 4352;  // >= (tz - 1) pz + (ty - 1) py + tx for every shape below

// Line tiles (FP32 3D): whole periodic x lines, so no x tap needs a test.
// Without the fused x pass (2N = 16) they hold 8 x 8 (y, z) rows in one
// 1024-thread block.
constexpr int kLineRows = 8;
constexpr int kLineBlock = 1024;

inline int line_pitch(int nf) { return nf + 11; }  // nf + 8 wrap slots, odd against bank aliasing of rows

// 2N in {32, 64, 128, 256}: line tiles with the fused x pass, 8 (y) x 4 (z)
// rows so that two blocks share a CU
inline bool fused_x_pass(int nf) { return nf >= 32 && nf <= 256; }
constexpr int kFusedRowsZ = 4;
constexpr int kFusedBlock = 512;

TileShape tile_shape(int nf, bool planar, bool line) {
    TileShape t{};
    if (line) {
        t.tx = nf;
        t.ty = kLineRows;
        t.tz = fused_x_pass(nf) ? kFusedRowsZ : kLineRows;
        t.ntx = 1;
        t.nty = nf / t.ty;
        t.ntz = nf / t.tz;
        t.py = line_pitch(nf);
        t.pz = t.ty * t.py;
        return t;
    }
    if (planar) {
        t.tx = nf < 64 ? nf : 64;
        t.ty = t.tx;
        t.tz = 1;
    } else {
        t.tx = nf < 32 ? nf : 32;
        t.ty = nf < 16 ? nf : 16;
        t.tz = nf < 8 ? nf : 8;
    }
    t.ntx = nf / t.tx;
    t.nty = nf / t.ty;
    t.ntz = planar ? 1 : nf / t.tz;
    // rows one node longer and planes three more: a rotated cluster of
    // samples then spreads over about twice as many banks
    t.py = t.tx + 1;
    t.pz = t.ty * t.py + 3;
    return t;
}

// first kernel node along an axis (not wrapped); the bin and tile kernels
// both take it from the same stored v
template <typename T>
__device__ __forceinline__ int first_node(T v, T half) {
    return int(dceil(v - half));
}

__global__ void clear_ints_kernel(int* __restrict__ p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0;
}

// SCATTER = false counts the samples of each (rotation, tile) bin; true
// writes each sample's fine position (4 reals) and coefficient at
// offsets[bin] + its rank in the bin (arrival order).  Zero samples are skipped.
template <typename T, int DIM, bool SCATTER>
__global__ __launch_bounds__(256) void nfft_bin_kernel(const T* __restrict__ pos, const cplx<T>* __restrict__ c,
                                                       int64_t m, const T* __restrict__ R, int nf, int w, TileShape ts,
                                                       int* __restrict__ counts, const int* __restrict__ offsets,
                                                       int* __restrict__ cursor, T* __restrict__ vbuf,
                                                       cplx<T>* __restrict__ cbuf) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int lane = int(threadIdx.x & 63);
    const int rot = int(blockIdx.y);
    cplx<T> ck = mk(T(0), T(0));
    if (k < m) ck = c[k];
    const bool active = k < m && (ck.re != T(0) || ck.im != T(0));
    T v[3] = {T(0), T(0), T(0)};
    int64_t bin = -1;
    if (active) {
        const T* r = R + 9 * rot;
        const T px = pos[3 * k], py = pos[3 * k + 1], pz = DIM == 3 ? pos[3 * k + 2] : T(0);
        const T fn = T(nf), half = T(0.5 * w);
        int b[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const T y = -T(2) * (r[3 * a] * px + r[3 * a + 1] * py + r[3 * a + 2] * pz);
            v[a] = y - dev_floor(y / fn) * fn;
            const int l0 = first_node(v[a], half);  // in [-w/2, nf)
            b[a] = l0 < 0 ? l0 + nf : l0;
        }
        const int nbins = ts.ntx * ts.nty * ts.ntz;
        bin = int64_t(rot) * nbins + (b[2] / ts.tz * ts.nty + b[1] / ts.ty) * ts.ntx + b[0] / ts.tx;
    }
    // Samples are in Morton order, so a wave's lanes share few bins: each
    // group of lanes with one bin makes one atomic, issued by its lowest lane.
    unsigned long long pending = __ballot(active);
    int64_t slot = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int64_t lbin = __shfl(bin, leader);
        const unsigned long long grp = __ballot(active && bin == lbin);
        const int cnt = __popcll(grp);
        if (!SCATTER) {
            if (lane == leader) atomicAdd(&counts[lbin], cnt);
        } else {
            int base = 0;
            if (lane == leader) base = offsets[lbin] + atomicAdd(&cursor[lbin], cnt);
            base = __shfl(base, leader);
            if ((grp >> lane) & 1ull) slot = int64_t(base) + __popcll(grp & ((1ull << lane) - 1ull));
        }
        pending &= ~grp;
    }
    if (SCATTER && active) {
        vbuf[4 * slot] = v[0];
        vbuf[4 * slot + 1] = v[1];
        vbuf[4 * slot + 2] = v[2];
        cbuf[slot] = ck;
    }
}

// Fixed-point accumulation of a tile: LDS integer atomics run many times
// faster than LDS float atomics.  Each tile takes its own scale from
// S = sum over the samples that touch it of max(|Re c|, |Im c|): every term
// c w (|w| <= 1) then maps to at most 2^30 (FP32, int32) or 2^62 (FP64,
// int64) in magnitude, and so does every partial sum, in any order.
template <typename T>
struct TileAcc;
template <>
struct TileAcc<float> {
    using A = int;
    static constexpr double kOne = 1073741824.0;  // 2^30
    __device__ static A to(float v) { return __float2int_rn(v); }
    __device__ static float back(int a) { return float(a); }
};
template <>
struct TileAcc<double> {
    using A = unsigned long long;  // two's complement sums, read back as signed
    static constexpr double kOne = 4611686018427387904.0;  // 2^62
    __device__ static A to(double v) { return (unsigned long long)__double2ll_rn(v); }
    __device__ static double back(unsigned long long a) { return double((long long)a); }
};

// S is taken without depending on the order of its terms: the bins list
// their samples in arrival order, so a floating-point sum would differ from
// run to run, and with it the scale and every fixed-point value of the tile.
// With M the block's largest term, each term t counts ceil(t 2^24 / M) units
// of M 2^-24, summed exactly in 64-bit integers (the rounding up keeps S at
// or above the exact sum, up to the final conversion's half ulp, which the
// 2x headroom of the accumulator covers).
template <typename T, int BS>
__device__ __forceinline__ T block_max_nonneg(T v, T* red) {
    for (int off = 32; off > 0; off >>= 1) {
        const T o = __shfl_xor(v, off);
        v = v > o ? v : o;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T m = red[0];
#pragma unroll
    for (int i = 1; i < BS / 64; ++i) m = m > red[i] ? m : red[i];
    return m;
}
template <int BS>
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long s = 0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) s += red[i];
    return s;
}
constexpr double kSumUnits = 16777216.0;  // 2^24 units per largest term
template <typename T>
__device__ __forceinline__ unsigned long long sum_units(T t, T per_unit) {
    return (unsigned long long)ceil(double(t * per_unit));
}

// offset o in (-2 nf, nf) of a node from a tile origin, wrapped to [0, nf)
__device__ __forceinline__ int wrap_offset(int o, int nf) {
    o += o < 0 ? nf : 0;
    o += o < 0 ? nf : 0;
    return o;
}
// node o + q < 2 nf wrapped to [0, nf)
__device__ __forceinline__ int wrap_once(int x, int nf) { return x >= nf ? x - nf : x; }

// per axis: do any of the W nodes ow + q (mod nf) fall in [0, side)?  ow is
// the wrapped offset of the first node
template <int W>
__device__ __forceinline__ bool reaches(int ow, int side, int nf) {
    bool hit = false;
#pragma unroll
    for (int q = 0; q < W; ++q) hit |= wrap_once(ow + q, nf) < side;
    return hit;
}

// One block per (tile, rotation): pass 1 sums S over the touching samples,
// pass 2 spreads them in fixed point, then every node of the tile is stored.
template <typename T, int DIM, int W>
__global__ __launch_bounds__(256) void nfft_tile_kernel(const T* __restrict__ vbuf, const cplx<T>* __restrict__ cbuf,
                                                        const int* __restrict__ counts, const int* __restrict__ offsets,
                                                        int nf, TileShape ts, cplx<T>* __restrict__ fine) {
    using Acc = TileAcc<T>;
    using A = typename Acc::A;
    __shared__ A lre[kTileLds], lim[kTileLds];
    __shared__ T red[4];
    __shared__ unsigned long long redi[4];
    const int nbins = ts.ntx * ts.nty * ts.ntz;
    const int tile = int(blockIdx.x), rot = int(blockIdx.y);
    const int tbx = tile % ts.ntx, tby = (tile / ts.ntx) % ts.nty, tbz = tile / (ts.ntx * ts.nty);
    const int org[3] = {tbx * ts.tx, tby * ts.ty, tbz * ts.tz};
    const int side[3] = {ts.tx, ts.ty, ts.tz};
    const int nodes = ts.tx * ts.ty * ts.tz;
    const T half = T(0.5 * W), beta = T(kEsBetaPerWidth * W), zs = T(2.0 / W);
    for (int e = int(threadIdx.x); e < kTileLds; e += 256) {
        lre[e] = A(0);
        lim[e] = A(0);
    }
    // the bins whose samples can reach this tile: its own and the ones just
    // below it along each axis that has more than one tile
    int bstart[8], bcount[8], nbs = 0;
    for (int nb = 0; nb < (1 << DIM); ++nb) {
        const int dx = nb & 1, dy = (nb >> 1) & 1, dz = (nb >> 2) & 1;
        if ((dx && ts.ntx == 1) || (dy && ts.nty == 1) || (dz && ts.ntz == 1)) continue;
        const int bx = (tbx - dx + ts.ntx) % ts.ntx, by = (tby - dy + ts.nty) % ts.nty;
        const int bz = (tbz - dz + ts.ntz) % ts.ntz;
        const int64_t bin = int64_t(rot) * nbins + (bz * ts.nty + by) * ts.ntx + bx;
        bstart[nbs] = offsets[bin];
        bcount[nbs] = counts[bin];
        ++nbs;
    }
    // pass 1: S, order-free (the largest term, then the sum in its units)
    auto terms = [&](auto&& take) __attribute__((always_inline)) {
        for (int bi = 0; bi < nbs; ++bi) {
            for (int p = int(threadIdx.x); p < bcount[bi]; p += 256) {
                const int64_t at = int64_t(bstart[bi]) + p;
                const T* vp = vbuf + 4 * at;
                bool hit = true;
#pragma unroll
                for (int a = 0; a < DIM; ++a)
                    hit = hit && reaches<W>(wrap_offset(first_node(vp[a], half) - org[a], nf), side[a], nf);
                if (hit) {
                    const cplx<T> ck = cbuf[at];
                    take(dmax(dabs(ck.re), dabs(ck.im)));
                }
            }
        }
    };
    T tmax = T(0);
    terms([&](T t) { tmax = t > tmax ? t : tmax; });
    const T M = block_max_nonneg<T, 256>(tmax, red);
    T S = T(0);
    if (M > T(0)) {
        const T per_unit = T(kSumUnits) / M;
        unsigned long long units = 0;
        terms([&](T t) { units += sum_units(t, per_unit); });
        S = T(double(block_sum_u64<256>(units, redi)) * (double(M) / kSumUnits));
    }
    const T sc = S > T(0) ? T(Acc::kOne) / S : T(0);
    // pass 2: spread in fixed point
    if (S > T(0)) {
        for (int bi = 0; bi < nbs; ++bi) {
            for (int p = int(threadIdx.x); p < bcount[bi]; p += 256) {
                const int64_t at = int64_t(bstart[bi]) + p;
                const T* vp = vbuf + 4 * at;
                int o[3] = {0, 0, 0}, l0[3] = {0, 0, 0};
                T va[3] = {T(0), T(0), T(0)};
                bool hit = true;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    va[a] = vp[a];
                    l0[a] = first_node(va[a], half);
                    o[a] = wrap_offset(l0[a] - org[a], nf);
                    hit = hit && reaches<W>(o[a], side[a], nf);
                }
                if (!hit) continue;
                const cplx<T> ck = cbuf[at];
                const T cre = ck.re * sc, cim = ck.im * sc;
                T wt[3][W];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const T z = (T(l0[a] + q) - va[a]) * zs;
                        const T sq = T(1) - z * z;
                        wt[a][q] = sq >= T(0) ? dexp(beta * (dsqrt(sq) - T(1))) : T(0);
                    }
                }
                if (DIM == 2) {
#pragma unroll
                    for (int bq = 0; bq < W; ++bq) {
                        const int iy = wrap_once(o[1] + bq, nf);
                        if (iy >= ts.ty) continue;
#pragma unroll
                        for (int aq = 0; aq < W; ++aq) {
                            const int ix = wrap_once(o[0] + aq, nf);
                            if (ix >= ts.tx) continue;
                            const T wgt = wt[0][aq] * wt[1][bq];
                            atomicAdd(&lre[iy * ts.py + ix], Acc::to(cre * wgt));
                            atomicAdd(&lim[iy * ts.py + ix], Acc::to(cim * wgt));
                        }
                    }
                } else {
#pragma unroll
                    for (int cq = 0; cq < W; ++cq) {
                        const int iz = wrap_once(o[2] + cq, nf);
                        if (iz >= ts.tz) continue;
#pragma unroll
                        for (int bq = 0; bq < W; ++bq) {
                            const int iy = wrap_once(o[1] + bq, nf);
                            if (iy >= ts.ty) continue;
                            const T wyz = wt[1][bq] * wt[2][cq];
                            const int rowo = iz * ts.pz + iy * ts.py;
#pragma unroll
                            for (int aq = 0; aq < W; ++aq) {
                                const int ix = wrap_once(o[0] + aq, nf);
                                if (ix >= ts.tx) continue;
                                const T wgt = wt[0][aq] * wyz;
                                atomicAdd(&lre[rowo + ix], Acc::to(cre * wgt));
                                atomicAdd(&lim[rowo + ix], Acc::to(cim * wgt));
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    const T inv = S > T(0) ? S / T(Acc::kOne) : T(0);
    const int64_t gsz = DIM == 3 ? int64_t(nf) * nf * nf : int64_t(nf) * nf;
    cplx<T>* g = fine + int64_t(rot) * gsz;
    for (int e = int(threadIdx.x); e < nodes; e += 256) {
        const int ix = e % ts.tx, iy = (e / ts.tx) % ts.ty, iz = e / (ts.tx * ts.ty);
        const int l = iz * ts.pz + iy * ts.py + ix;
        g[(int64_t(org[2] + iz) * nf + (org[1] + iy)) * nf + (org[0] + ix)] = mk(Acc::back(lre[l]) * inv, Acc::back(lim[l]) * inv);
    }
}

// ------------------------------------------------------------------ pruned transform
// Forward FFT of the 2N grid that keeps only the N central modes per axis:
// each pass transforms full 2N-point lines in LDS and stores the N kept
// outputs, so the next pass reads half as much (x: 2N^3 -> N (2N)^2 values,
// y: -> N^2 2N, z: -> N^3).  The last pass divides by the kernel's transform
// and multiplies by the fixed spectrum.

// j-th of the N kept modes (FFT order) on the 2N grid
__device__ __forceinline__ int fine_mode(int j, int N) { return j < N / 2 ? j : j + N; }

template <typename T, int NF>
__global__ __launch_bounds__(256) void nfft_rows_pruned_kernel(const cplx<T>* __restrict__ in,
                                                               cplx<T>* __restrict__ out, int64_t nrows) {
    constexpr int TPL = FFTShape<NF>::TPL, CONC = 256 / TPL, N = NF / 2;
    __shared__ cplx<T> buf[CONC * NF];
    __shared__ cplx<T> tw[NF];
    fill_twiddles<T, NF>(tw);
    const int64_t row0 = int64_t(blockIdx.x) * CONC;
    const int nr = int(nrows - row0 < CONC ? nrows - row0 : CONC);
    const cplx<T>* src = in + row0 * NF;
    for (int i = int(threadIdx.x); i < nr * NF; i += 256) buf[i] = src[i];
    __syncthreads();
    lds_fft_lines<T, NF, -1, false>(buf, 1, NF, nr, tw);
    cplx<T>* dst = out + row0 * N;
    for (int i = int(threadIdx.x); i < nr * N; i += 256) {
        const int r = i / N, j = i - r * N;
        dst[i] = buf[r * NF + fine_mode(j, N)];
    }
}

// columns per block: a power of two that the block's threads cover and that
// divides N
template <int NF, int BS = 256>
constexpr int pruned_width() {
    int w = 1;
    while (w * 2 <= BS / FFTShape<NF>::TPL && w * 2 <= NF / 2) w *= 2;
    return w;
}

// threads per column block: 512 for 2N = 256, so a block reads 16 columns
// (128-byte row segments) instead of 8
template <int NF>
constexpr int cols_block() {
    return NF >= 256 ? 512 : 256;
}

// A block transforms W consecutive x columns along a strided axis (element
// stride es_in) and stores the N kept outputs (stride es_out).  FINAL: the
// axis is the last one (y of a planar grid, z in 3D); outputs are the modes
// (jx, jy[, jz]) times inv[jx] inv[jy] [inv[jz]] spec.
// TILED (FINAL, 3D, N = 64 or 128): outputs go to column tiles with
// pair-grouped positions, the layout the search path's pencil pass reads
template <typename T, int NF, bool FINAL, bool PLANAR, int BS = cols_block<NF>(), bool TILED = false>
__global__ __launch_bounds__(BS) void nfft_cols_pruned_kernel(const cplx<T>* __restrict__ in,
                                                               cplx<T>* __restrict__ out, int64_t es_in,
                                                               int64_t os_in, int64_t bs_in, int64_t es_out,
                                                               int64_t os_out, int64_t bs_out,
                                                               const T* __restrict__ inv,
                                                               const cplx<T>* __restrict__ spec) {
    constexpr int W = pruned_width<NF, BS>(), N = NF / 2;
    __shared__ cplx<T> buf[NF * W];
    __shared__ cplx<T> tw[NF];
    fill_twiddles<T, NF>(tw);
    const int x0 = int(blockIdx.x) * W, o = int(blockIdx.y), b = int(blockIdx.z);
    const cplx<T>* src = in + int64_t(b) * bs_in + int64_t(o) * os_in + x0;
    for (int i = int(threadIdx.x); i < NF * W; i += BS) {
        const int e = i / W, xl = i - e * W;
        buf[i] = src[int64_t(e) * es_in + xl];
    }
    __syncthreads();
    lds_fft_lines<T, NF, -1, true>(buf, W, 1, W, tw);
    cplx<T>* dst = out + int64_t(b) * bs_out + int64_t(o) * os_out + x0;
    for (int i = int(threadIdx.x); i < N * W; i += BS) {
        const int j = i / W, xl = i - j * W;
        cplx<T> v = buf[fine_mode(j, N) * W + xl];
        if (FINAL) {
            const int jx = x0 + xl, jy = PLANAR ? j : o, jz = PLANAR ? 0 : j;
            const T sc = inv[jx] * inv[jy] * (PLANAR ? T(1) : inv[jz]);
            v = v * sc * spec[(int64_t(jz) * N + jy) * N + jx];
        }
        if constexpr (TILED) {
            static_assert(FINAL && !PLANAR && (N == 64 || N == 128), "column tiles: 3D, N = 64 or 128");
            out[int64_t(b) * bs_out + tile_index<N>(j, o, col_pos<N>(x0 + xl))] = v;
        } else {
            dst[int64_t(j) * es_out + xl] = v;
        }
    }
}

// rows_done: the x pass already wrote half_buf (fused into the line tiles)
template <typename T, int NF>
void pruned_transform(const cplx<T>* fine, cplx<T>* half_buf, cplx<T>* quarter_buf, int batch, bool planar,
                      const T* inv, const cplx<T>* spec, cplx<T>* out, bool rows_done, bool tiled, hipStream_t s) {
    constexpr int N = NF / 2, TPL = FFTShape<NF>::TPL, CONC = 256 / TPL, BS = cols_block<NF>(),
                  W = pruned_width<NF, BS>();
    const int64_t nrows = int64_t(batch) * NF * (planar ? 1 : NF);
    if (!rows_done)
        hipLaunchKernelGGL((nfft_rows_pruned_kernel<T, NF>), dim3(unsigned((nrows + CONC - 1) / CONC)), dim3(256),
                           0, s, fine, half_buf, nrows);
    if (planar) {
        // y, last: half_buf [b][y < NF][x < N] -> out [b][jy][jx]
        hipLaunchKernelGGL((nfft_cols_pruned_kernel<T, NF, true, true>), dim3(N / W, 1, unsigned(batch)), dim3(BS),
                           0, s, half_buf, out, int64_t(N), int64_t(0), int64_t(NF) * N, int64_t(N), int64_t(0),
                           int64_t(N) * N, inv, spec);
        return;
    }
    // y: half_buf [b][z < NF][y < NF][x < N] -> quarter_buf [b][z < NF][jy][x < N]
    hipLaunchKernelGGL((nfft_cols_pruned_kernel<T, NF, false, false>), dim3(N / W, NF, unsigned(batch)), dim3(BS),
                       0, s, half_buf, quarter_buf, int64_t(N), int64_t(NF) * N, int64_t(NF) * NF * N, int64_t(N),
                       int64_t(N) * N, int64_t(NF) * N * N, inv, spec);
    // z, last: quarter_buf [b][z < NF][jy][jx] -> out [b][jz][jy][jx] (or column tiles)
    if constexpr (NF == 128 || NF == 256) {
        if (tiled) {
            hipLaunchKernelGGL((nfft_cols_pruned_kernel<T, NF, true, false, BS, true>), dim3(N / W, N, unsigned(batch)),
                               dim3(BS), 0, s, quarter_buf, out, int64_t(N) * N, int64_t(N), int64_t(NF) * N * N,
                               int64_t(N) * N, int64_t(N), int64_t(N) * N * N, inv, spec);
            return;
        }
    }
    hipLaunchKernelGGL((nfft_cols_pruned_kernel<T, NF, true, false>), dim3(N / W, N, unsigned(batch)), dim3(BS), 0,
                       s, quarter_buf, out, int64_t(N) * N, int64_t(N), int64_t(NF) * N * N, int64_t(N) * N,
                       int64_t(N), int64_t(N) * N * N, inv, spec);
}

template <typename T>
hipError_t launch_pruned(const cplx<T>* fine, cplx<T>* half_buf, cplx<T>* quarter_buf, int batch, int N, bool planar,
                         const T* inv, const cplx<T>* spec, cplx<T>* out, bool rows_done, bool tiled, hipStream_t s) {
    switch (2 * N) {
#define SDF_PRUNED(NF)                                                                                             \
    case NF:                                                                                                       \
        pruned_transform<T, NF>(fine, half_buf, quarter_buf, batch, planar, inv, spec, out, rows_done, tiled, s);   \
        break;
        SDF_PRUNED(16)
        SDF_PRUNED(32)
        SDF_PRUNED(64)
        SDF_PRUNED(128)
        SDF_PRUNED(192)
        SDF_PRUNED(256)
#undef SDF_PRUNED
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Line tile without the fused transform (FP32, 3D, 2N = 16): one block per
// (8 x 8 rows of whole x lines, rotation).
// Samples of the tile's bin and of the bins below it in y and z; per
// sample, each of its W^2 (y, z) rows that lies in the tile is one branch
// with W unconditional integer adds at constant offsets from the row base
// (x positions past the line's end land in 8 spare slots, folded back when
// the row is stored).  Fixed-point scale per tile as in nfft_tile_kernel.
constexpr int kLineLds = kLineRows * kLineRows * (256 + 11);  // ints per plane at nf = 256

template <int W>
__global__ __launch_bounds__(kLineBlock) void nfft_line_tile_kernel(const float* __restrict__ vbuf,
                                                                    const cplx<float>* __restrict__ cbuf,
                                                                    const int* __restrict__ counts,
                                                                    const int* __restrict__ offsets, int nf,
                                                                    TileShape ts, cplx<float>* __restrict__ fine) {
    __shared__ int lre[kLineLds], lim[kLineLds];
    __shared__ float red[kLineBlock / 64];
    __shared__ unsigned long long redi[kLineBlock / 64];
    const int nbins = ts.nty * ts.ntz;
    const int tile = int(blockIdx.x), rot = int(blockIdx.y);
    const int tby = tile % ts.nty, tbz = tile / ts.nty;
    const int y0 = tby * kLineRows, z0 = tbz * kLineRows;
    const int px = ts.py;
    const int used = kLineRows * kLineRows * px;
    const int msk = nf - 1;
    const float half = float(0.5 * W), beta = float(kEsBetaPerWidth * W), zs = float(2.0 / W);
    int bstart[4], bcount[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int by = (tby - (nb & 1) + ts.nty) % ts.nty, bz = (tbz - (nb >> 1) + ts.ntz) % ts.ntz;
        const int64_t bin = int64_t(rot) * nbins + bz * ts.nty + by;
        bstart[nb] = offsets[bin];
        bcount[nb] = counts[bin];
    }
    // y / z offset of a sample's first window row from the tile, in (-nf/2, nf/2]
    auto rel = [&](float v, int org) { return ((first_node(v, half) - org + nf / 2) & msk) - nf / 2; };
    auto terms = [&](auto&& take) __attribute__((always_inline)) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            for (int p = int(threadIdx.x); p < bcount[nb]; p += kLineBlock) {
                const int64_t at = int64_t(bstart[nb]) + p;
                const float* vp = vbuf + 4 * at;
                const int oy = rel(vp[1], y0), oz = rel(vp[2], z0);
                if (oy > -W && oy < kLineRows && oz > -W && oz < kLineRows) {
                    const cplx<float> ck = cbuf[at];
                    take(fmaxf(fabsf(ck.re), fabsf(ck.im)));
                }
            }
        }
    };
    float tmax = 0.f;
    terms([&](float t) { tmax = fmaxf(tmax, t); });
    const float M = block_max_nonneg<float, kLineBlock>(tmax, red);
    float S = 0.f;
    if (M > 0.f) {
        const float per_unit = float(kSumUnits) / M;
        unsigned long long units = 0;
        terms([&](float t) { units += sum_units(t, per_unit); });
        S = float(double(block_sum_u64<kLineBlock>(units, redi)) * (double(M) / kSumUnits));
    }
    cplx<float>* g = fine + int64_t(rot) * nf * nf * nf;
    const int sh = __ffs(nf) - 1;  // nf is a power of two
    if (!(S > 0.f)) {  // no sample reaches the tile: store zeros, skip the LDS work
        for (int e = int(threadIdx.x); e < kLineRows * kLineRows * nf; e += kLineBlock) {
            const int x = e & msk, row = e >> sh;
            g[(int64_t(z0 + row / kLineRows) * nf + (y0 + row % kLineRows)) * nf + x] = mk(0.f, 0.f);
        }
        return;
    }
    for (int e = int(threadIdx.x); e < used; e += kLineBlock) {
        lre[e] = 0;
        lim[e] = 0;
    }
    __syncthreads();
    const float sc = float(TileAcc<float>::kOne) / S;
    {
#pragma unroll 1
        for (int nb = 0; nb < 4; ++nb) {
            for (int p = int(threadIdx.x); p < bcount[nb]; p += kLineBlock) {
                const int64_t at = int64_t(bstart[nb]) + p;
                const float* vp = vbuf + 4 * at;
                const float vx = vp[0], vy = vp[1], vz = vp[2];
                const int oy = rel(vy, y0), oz = rel(vz, z0);
                if (!(oy > -W && oy < kLineRows && oz > -W && oz < kLineRows)) continue;
                const int lx = first_node(vx, half);
                const int ly = first_node(vy, half), lz = first_node(vz, half);
                const cplx<float> ck = cbuf[at];
                float xr[W], xi[W], wy[W], wz[W];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const float zx = (float(lx + q) - vx) * zs, zy = (float(ly + q) - vy) * zs,
                                zz = (float(lz + q) - vz) * zs;
                    const float sx = 1.f - zx * zx, sy = 1.f - zy * zy, sz = 1.f - zz * zz;
                    const float wx = sx >= 0.f ? expf(beta * (sqrtf(sx) - 1.f)) : 0.f;
                    wy[q] = sy >= 0.f ? expf(beta * (sqrtf(sy) - 1.f)) : 0.f;
                    wz[q] = sz >= 0.f ? expf(beta * (sqrtf(sz) - 1.f)) : 0.f;
                    xr[q] = ck.re * sc * wx;
                    xi[q] = ck.im * sc * wx;
                }
                const int xb = lx & msk;  // taps xb .. xb + W - 1 < nf + 8
#pragma unroll
                for (int cq = 0; cq < W; ++cq) {
                    const int iz = oz + cq;
#pragma unroll
                    for (int bq = 0; bq < W; ++bq) {
                        const int iy = oy + bq;
                        if (unsigned(iz) < unsigned(kLineRows) && unsigned(iy) < unsigned(kLineRows)) {
                            const float wyz = wy[bq] * wz[cq];
                            int* rr = lre + (iz * kLineRows + iy) * px + xb;
                            int* ri = lim + (iz * kLineRows + iy) * px + xb;
#pragma unroll
                            for (int aq = 0; aq < W; ++aq) {
                                atomicAdd(rr + aq, __float2int_rn(xr[aq] * wyz));
                                atomicAdd(ri + aq, __float2int_rn(xi[aq] * wyz));
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    const float inv = S / float(TileAcc<float>::kOne);
    for (int e = int(threadIdx.x); e < kLineRows * kLineRows * nf; e += kLineBlock) {
        const int x = e & msk, row = e >> sh;  // row = iz * 8 + iy
        const int iy = row % kLineRows, iz = row / kLineRows;
        int ar = lre[row * px + x], ai = lim[row * px + x];
        if (x < 8) {  // fold the wrap slots
            ar += lre[row * px + nf + x];
            ai += lim[row * px + nf + x];
        }
        g[(int64_t(z0 + iz) * nf + (y0 + iy)) * nf + x] = mk(float(ar) * inv, float(ai) * inv);
    }
}

template <int W>
void launch_line_tile(const float* vbuf, const cplx<float>* cbuf, const int* counts, const int* offsets, int batch,
                      int nf, TileShape ts, cplx<float>* fine, hipStream_t s) {
    hipLaunchKernelGGL((nfft_line_tile_kernel<W>), dim3(unsigned(ts.nty * ts.ntz), unsigned(batch)),
                       dim3(kLineBlock), 0, s, vbuf, cbuf, counts, offsets, nf, ts, fine);
}

// Line tile with the x pass of the pruned transform fused in (FP32, 3D,
// 2N >= 32): 8 (y) x 4 (z) rows of whole x lines, 512 threads and 77 KiB of
// LDS (67 KiB of integer rows, the 256 twiddles, the candidate sort's
// histogram and 8 KiB of sorted indices), so two blocks share a CU and
// overlap their phases.  A window of w
// nodes reaches 1 + ceil((w - 1) / 4) z tiles, so the tile gathers the bins
// of its own (y, z) and of the next one below in y and up to two below in z.
// After the fixed-point accumulation the 32 x lines are converted to complex
// in the same LDS, transformed there (2N points), and only the N kept modes
// of each line are stored, into the x-pruned buffer [b][z][y][N] that the y
// pass reads.  The oversampled grid itself is never written to memory.
constexpr int kFusedRows = kLineRows * kFusedRowsZ;
constexpr int kFusedLds = kFusedRows * (256 + 11);  // ints per plane at nf = 256

template <int W, int NF>
__global__ __launch_bounds__(kFusedBlock) void nfft_line_fft_kernel(const float* __restrict__ vbuf,
                                                                    const cplx<float>* __restrict__ cbuf,
                                                                    const int* __restrict__ counts,
                                                                    const int* __restrict__ offsets, TileShape ts,
                                                                    cplx<float>* __restrict__ half_buf) {
    constexpr int nf = NF, N = NF / 2, msk = NF - 1, RY = kLineRows, RZ = kFusedRowsZ, ROWS = kFusedRows;
    constexpr int BS = kFusedBlock;
    constexpr int PER = ROWS * NF / BS;  // converted values per thread
    constexpr int NBZ = 1 + (W - 1 + RZ - 1) / RZ, NB = 2 * NBZ;
    static_assert(ROWS * NF * sizeof(cplx<float>) <= 2 * kFusedLds * sizeof(int), "complex rows exceed the LDS");
    __shared__ __align__(16) int acc[2 * kFusedLds];
    __shared__ cplx<float> tw[NF];
    __shared__ float red[BS / 64];
    __shared__ unsigned long long redi[BS / 64];
    // counting sort of the touching candidates by (z, y) row offset: oy in
    // (-W, 8), oz in (-W, 4), W <= 8
    constexpr int KEYS = 15 * 11;
    // each thread keeps its first KC candidates in registers (and the sort
    // covers those KC * BS); later ones are spread unsorted
    constexpr int KC = 4;
    __shared__ int s_hist[KEYS];
    __shared__ int s_idx[KC * BS];
    __shared__ int s_nsorted;
    // two blocks share a compute unit's 160 KiB only while one stays within 80 KiB
    static_assert(sizeof(int) * (2 * kFusedLds + KEYS + KC * BS + 1) + sizeof(cplx<float>) * NF +
                          (sizeof(float) + sizeof(unsigned long long)) * (BS / 64) <= 80 * 1024,
                  "the fused line tile must fit two blocks per compute unit");
    int* lre = acc;
    int* lim = acc + kFusedLds;
    cplx<float>* cb = reinterpret_cast<cplx<float>*>(acc);
    fill_twiddles<float, NF>(tw);
    const int nbins = ts.nty * ts.ntz;
    const int tile = int(blockIdx.x), rot = int(blockIdx.y);
    const int tby = tile % ts.nty, tbz = tile / ts.nty;
    const int y0 = tby * RY, z0 = tbz * RZ;
    const int px = ts.py;
    const float half = float(0.5 * W), beta = float(kEsBetaPerWidth * W), zs = float(2.0 / W);
    // candidates: the bins (tby - dy, tbz - dz), dy < 2, dz < NBZ, as one flat
    // list; each thread keeps its first KC in registers from the S pass to the
    // spreading pass (their loads issue together)
    int bstart[NB], bpre[NB + 1];
    bpre[0] = 0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int by = (tby - (nb & 1) + ts.nty) % ts.nty, bz = (tbz - (nb >> 1) + ts.ntz) % ts.ntz;
        const int64_t bin = int64_t(rot) * nbins + bz * ts.nty + by;
        bstart[nb] = offsets[bin];
        bpre[nb + 1] = bpre[nb] + counts[bin];
    }
    const int total = bpre[NB];
    // base of candidate i's bin minus the candidates before it: the bin
    // boundaries are ordered, so the deltas of the passed ones add up
    int delta[NB];
    delta[0] = bstart[0];
#pragma unroll
    for (int nb = 1; nb < NB; ++nb) delta[nb] = (bstart[nb] - bpre[nb]) - (bstart[nb - 1] - bpre[nb - 1]);
    auto slot = [=](int i) __attribute__((always_inline)) {
        int base = delta[0];
#pragma unroll
        for (int nb = 1; nb < NB; ++nb) base += int(i >= bpre[nb]) * delta[nb];
        return int64_t(base) + i;
    };
    // x in (-nf, 2 nf) wrapped to [0, nf)
    auto wrapnf = [](int x) __attribute__((always_inline)) {
        if constexpr ((NF & (NF - 1)) == 0) {
            return x & msk;
        } else {
            x += x < 0 ? NF : 0;
            return x >= NF ? x - NF : x;
        }
    };
    auto rel = [=](float v, int org) __attribute__((always_inline)) {
        return wrapnf(first_node(v, half) - org + nf / 2) - nf / 2;
    };
    auto touches = [=](int oy, int oz) __attribute__((always_inline)) {
        return oy > -W && oy < RY && oz > -W && oz < RZ;
    };
    float cvx[KC], cvy[KC], cvz[KC];
    cplx<float> cck[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int i = int(threadIdx.x) + k * BS;
        cvx[k] = cvy[k] = cvz[k] = 0.f;
        cck[k] = mk(0.f, 0.f);
        if (i < total) {
            const int64_t at = slot(i);
            cvx[k] = vbuf[4 * at];
            cvy[k] = vbuf[4 * at + 1];
            cvz[k] = vbuf[4 * at + 2];
            cck[k] = cbuf[at];
        }
    }
    // S, order-free: the largest term, then the sum in its units (the first
    // KC candidates of each thread from registers, the rest reloaded)
    auto terms = [&](auto&& take) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int i = int(threadIdx.x) + k * BS;
            if (i < total && touches(rel(cvy[k], y0), rel(cvz[k], z0))) take(fmaxf(fabsf(cck[k].re), fabsf(cck[k].im)));
        }
        for (int i = int(threadIdx.x) + KC * BS; i < total; i += BS) {
            const int64_t at = slot(i);
            if (touches(rel(vbuf[4 * at + 1], y0), rel(vbuf[4 * at + 2], z0))) {
                const cplx<float> ck = cbuf[at];
                take(fmaxf(fabsf(ck.re), fabsf(ck.im)));
            }
        }
    };
    float tmax = 0.f;
    terms([&](float t) { tmax = fmaxf(tmax, t); });
    const float M = block_max_nonneg<float, BS>(tmax, red);
    float S = 0.f;
    if (M > 0.f) {
        const float per_unit = float(kSumUnits) / M;
        unsigned long long units = 0;
        terms([&](float t) { units += sum_units(t, per_unit); });
        S = float(double(block_sum_u64<BS>(units, redi)) * (double(M) / kSumUnits));
    }
    // x-pruned rows of this tile: row r = iz * 8 + iy at [b][z0 + iz][y0 + iy][0 .. N)
    cplx<float>* hb = half_buf + int64_t(rot) * NF * NF * N;
    auto hrow = [=](int r) __attribute__((always_inline)) {
        return hb + (int64_t(z0 + r / RY) * NF + (y0 + r % RY)) * N;
    };
    if (!(S > 0.f)) {  // no sample reaches the tile: its modes are zero
        for (int e = int(threadIdx.x); e < ROWS * N; e += BS) hrow(e / N)[e % N] = mk(0.f, 0.f);
        return;
    }
    const int used = ROWS * px;
    for (int e = int(threadIdx.x); e < used; e += BS) {
        lre[e] = 0;
        lim[e] = 0;
    }
    for (int e = int(threadIdx.x); e < KEYS; e += BS) s_hist[e] = 0;
    __syncthreads();
    // Sort the register-held candidates that touch the tile by (oz, oy), so a
    // wave's lanes mostly share which of the window's rows lie in the tile and
    // the row branches run with full waves (the integer sums do not depend on
    // the order).
    int key[KC], rank[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        key[k] = -1;
        rank[k] = 0;
        if (int(threadIdx.x) + k * BS < total) {
            const int oy = rel(cvy[k], y0), oz = rel(cvz[k], z0);
            if (touches(oy, oz)) {
                key[k] = (oz + 7) * 15 + (oy + 7);
                rank[k] = atomicAdd(&s_hist[key[k]], 1);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {  // exclusive scan of the 165 bucket sizes, 3 per lane
        const int ln = int(threadIdx.x);
        const int v0 = 3 * ln < KEYS ? s_hist[3 * ln] : 0, v1 = 3 * ln + 1 < KEYS ? s_hist[3 * ln + 1] : 0,
                  v2 = 3 * ln + 2 < KEYS ? s_hist[3 * ln + 2] : 0;
        const int sum = v0 + v1 + v2;
        int incl = sum;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off);
            if (ln >= off) incl += t;
        }
        const int excl = incl - sum;
        if (3 * ln < KEYS) s_hist[3 * ln] = excl;
        if (3 * ln + 1 < KEYS) s_hist[3 * ln + 1] = excl + v0;
        if (3 * ln + 2 < KEYS) s_hist[3 * ln + 2] = excl + v0 + v1;
        if (ln == 63) s_nsorted = incl;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KC; ++k)
        if (key[k] >= 0) s_idx[s_hist[key[k]] + rank[k]] = int(threadIdx.x) + k * BS;
    __syncthreads();
    const int nsorted = s_nsorted;
    // the sorted candidates, reloaded (from L2) KC per thread
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int so = int(threadIdx.x) + k * BS;
        if (so < nsorted) {
            const int64_t at = slot(s_idx[so]);
            cvx[k] = vbuf[4 * at];
            cvy[k] = vbuf[4 * at + 1];
            cvz[k] = vbuf[4 * at + 2];
            cck[k] = cbuf[at];
        }
    }
    const float sc = float(TileAcc<float>::kOne) / S;
    auto spread = [=](float vx, float vy, float vz, cplx<float> ck) __attribute__((always_inline)) {
        const int oy = rel(vy, y0), oz = rel(vz, z0);
        if (!touches(oy, oz)) return;
        const int lx = first_node(vx, half);
        const int ly = first_node(vy, half), lz = first_node(vz, half);
        float xr[W], xi[W], wy[W], wz[W];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const float zx = (float(lx + q) - vx) * zs, zy = (float(ly + q) - vy) * zs, zz = (float(lz + q) - vz) * zs;
            const float sx = 1.f - zx * zx, sy = 1.f - zy * zy, sz = 1.f - zz * zz;
            const float wx = sx >= 0.f ? expf(beta * (sqrtf(sx) - 1.f)) : 0.f;
            wy[q] = sy >= 0.f ? expf(beta * (sqrtf(sy) - 1.f)) : 0.f;
            wz[q] = sz >= 0.f ? expf(beta * (sqrtf(sz) - 1.f)) : 0.f;
            xr[q] = ck.re * sc * wx;
            xi[q] = ck.im * sc * wx;
        }
        const int xb = wrapnf(lx);  // taps xb .. xb + W - 1 < nf + 8
#pragma unroll
        for (int cq = 0; cq < W; ++cq) {
            const int iz = oz + cq;
#pragma unroll
            for (int bq = 0; bq < W; ++bq) {
                const int iy = oy + bq;
                if (unsigned(iz) < unsigned(RZ) && unsigned(iy) < unsigned(RY)) {
                    const float wyz = wy[bq] * wz[cq];
                    int* rr = lre + (iz * RY + iy) * px + xb;
                    int* ri = lim + (iz * RY + iy) * px + xb;
#pragma unroll
                    for (int aq = 0; aq < W; ++aq) {
                        atomicAdd(rr + aq, __float2int_rn(xr[aq] * wyz));
                        atomicAdd(ri + aq, __float2int_rn(xi[aq] * wyz));
                    }
                }
            }
        }
    };
    // one copy of the spreading code: take element 0, then shift the register
    // copies down (constant indices keep them out of scratch)
#pragma unroll 1
    for (int k = 0; k < KC; ++k) {
        if (int(threadIdx.x) + k * BS < nsorted) spread(cvx[0], cvy[0], cvz[0], cck[0]);
#pragma unroll
        for (int j = 0; j + 1 < KC; ++j) {
            cvx[j] = cvx[j + 1];
            cvy[j] = cvy[j + 1];
            cvz[j] = cvz[j + 1];
            cck[j] = cck[j + 1];
        }
    }
    for (int i = int(threadIdx.x) + KC * BS; i < total; i += BS) {
        const int64_t at = slot(i);
        spread(vbuf[4 * at], vbuf[4 * at + 1], vbuf[4 * at + 2], cbuf[at]);
    }
    __syncthreads();
    // integer rows (with their wrap slots folded) -> complex lines in the same LDS
    const float inv = S / float(TileAcc<float>::kOne);
    cplx<float> val[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = int(threadIdx.x) + k * BS;
        const int x = e % NF, row = e / NF;
        int ar = lre[row * px + x], ai = lim[row * px + x];
        if (x < 8) {
            ar += lre[row * px + nf + x];
            ai += lim[row * px + nf + x];
        }
        val[k] = mk(float(ar) * inv, float(ai) * inv);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) cb[int(threadIdx.x) + k * BS] = val[k];
    __syncthreads();
    lds_fft_lines<float, NF, -1, false>(cb, 1, NF, ROWS, tw);
    __syncthreads();
    for (int e = int(threadIdx.x); e < ROWS * N; e += BS) {
        const int r = e / N, j = e % N;
        hrow(r)[j] = cb[r * NF + fine_mode(j, N)];
    }
}

template <int NF>
void launch_line_fft_nf(const float* vbuf, const cplx<float>* cbuf, const int* counts, const int* offsets, int batch,
                        int w, TileShape ts, cplx<float>* half_buf, hipStream_t s) {
    const dim3 grid(unsigned(ts.nty * ts.ntz), unsigned(batch));
    switch (w) {
#define SDF_LINE_W(WW)                                                                                          \
    case WW:                                                                                                    \
        hipLaunchKernelGGL((nfft_line_fft_kernel<WW, NF>), grid, dim3(kFusedBlock), 0, s, vbuf, cbuf, counts,  \
                           offsets, ts, half_buf);                                                              \
        break;
        SDF_LINE_W(2)
        SDF_LINE_W(3)
        SDF_LINE_W(4)
        SDF_LINE_W(5)
        SDF_LINE_W(6)
        SDF_LINE_W(7)
        SDF_LINE_W(8)
#undef SDF_LINE_W
        default: break;
    }
}

hipError_t launch_line_fft(const float* vbuf, const cplx<float>* cbuf, const int* counts, const int* offsets,
                           int batch, int nf, int w, TileShape ts, cplx<float>* half_buf, hipStream_t s) {
    if (w < 2 || w > 8) return hipErrorInvalidValue;
    switch (nf) {
        case 32: launch_line_fft_nf<32>(vbuf, cbuf, counts, offsets, batch, w, ts, half_buf, s); break;
        case 64: launch_line_fft_nf<64>(vbuf, cbuf, counts, offsets, batch, w, ts, half_buf, s); break;
        case 128: launch_line_fft_nf<128>(vbuf, cbuf, counts, offsets, batch, w, ts, half_buf, s); break;
        case 192: launch_line_fft_nf<192>(vbuf, cbuf, counts, offsets, batch, w, ts, half_buf, s); break;
        case 256: launch_line_fft_nf<256>(vbuf, cbuf, counts, offsets, batch, w, ts, half_buf, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int DIM>
hipError_t tile_width(const T* vbuf, const cplx<T>* cbuf, const int* counts, const int* offsets, int batch, int nf,
                      int w, TileShape ts, cplx<T>* fine, hipStream_t s) {
    const dim3 grid(unsigned(ts.ntx * ts.nty * ts.ntz), unsigned(batch));
    switch (w) {
#define SDF_NFFT_W(WW)                                                                                         \
    case WW:                                                                                                   \
        hipLaunchKernelGGL((nfft_tile_kernel<T, DIM, WW>), grid, dim3(256), 0, s, vbuf, cbuf, counts, offsets, \
                           nf, ts, fine);                                                                      \
        break;
        SDF_NFFT_W(2)
        SDF_NFFT_W(3)
        SDF_NFFT_W(4)
        SDF_NFFT_W(5)
        SDF_NFFT_W(6)
        SDF_NFFT_W(7)
        SDF_NFFT_W(8)
#undef SDF_NFFT_W
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// workspace of launch_nfft_modes: bin counts, cursors and offsets per
// (rotation, tile), the binned samples (4 + 2 reals each), scan temporaries
struct NfftWs {
    size_t counts, cursor, offsets, vbuf, cbuf, half, temp, temp_bytes, total;
};

// FP32 3D grids use line tiles; FP64 (whose 64-bit rows would not fit) and
// planar grids the general tiles
bool use_lines(bool planar, size_t elem) { return !planar && elem == sizeof(float); }

NfftWs nfft_ws_layout(int64_t m, int batch, int N, bool planar, size_t elem) {
    const TileShape ts = tile_shape(2 * N, planar, use_lines(planar, elem));
    const int64_t nb = int64_t(ts.ntx) * ts.nty * ts.ntz * batch;
    const size_t temp_bytes = scan_temp_bytes(int(nb));
    const size_t nbi = size_t(nb) * sizeof(int), ns = size_t(m) * size_t(batch);
    NfftWs L{};
    size_t off = 0;
    L.counts = off;
    off += (nbi + 255) / 256 * 256;
    L.cursor = off;
    off += (nbi + 255) / 256 * 256;
    L.offsets = off;
    off += (nbi + 255) / 256 * 256;
    L.vbuf = off;
    off += (4 * elem * ns + 255) / 256 * 256;
    L.cbuf = off;
    off += (2 * elem * ns + 255) / 256 * 256;
    // x-pruned transform: N (2N)^2 (planar N 2N) values per rotation
    const size_t hv = size_t(N) * 2 * N * (planar ? 1 : 2 * N) * size_t(batch);
    L.half = off;
    off += (2 * elem * hv + 255) / 256 * 256;
    L.temp = off;
    L.temp_bytes = temp_bytes;
    off += (temp_bytes + 255) / 256 * 256;
    L.total = off;
    return L;
}

// workspace of launch_octree: coefficients, A, per-block counts and
// offsets, scan temporaries
struct OctWs {
    size_t coef, amax, counts, offsets, temp, temp_bytes, total;
};

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

OctWs oct_ws_layout(int nm, bool planar, size_t elem) {
    const int64_t K = planar ? int64_t(nm) * nm : int64_t(nm) * nm * nm;
    const int nblk = int(K / (planar ? 64 : 512));
    const size_t temp_bytes = scan_temp_bytes(nblk);
    OctWs L{};
    size_t off = 0;
    L.coef = off;
    off += al256(2 * elem * size_t(K));
    L.amax = off;
    off += 256;
    L.counts = off;
    off += al256(sizeof(int) * size_t(nblk));
    L.offsets = off;
    off += al256(sizeof(int) * size_t(nblk));
    L.temp = off;
    L.temp_bytes = temp_bytes;
    off += al256(temp_bytes);
    L.total = off;
    return L;
}

}  // namespace

size_t octree_workspace_bytes(int nm, bool planar, size_t elem) { return oct_ws_layout(nm, planar, elem).total; }

template <typename T>
hipError_t launch_octree(const void* rho_m, const T* w_m, int nm, bool planar, double tol, int max_level, T* pos,
                         void* c_out, int* level, int64_t* count_out, void* ws, hipStream_t s) {
    using U = typename UBits<T>::U;
    const OctWs L = oct_ws_layout(nm, planar, sizeof(T));
    char* base = static_cast<char*>(ws);
    const int64_t K = planar ? int64_t(nm) * nm : int64_t(nm) * nm * nm;
    const int nblk = int(K / (planar ? 64 : 512));
    cplx<T>* coef = reinterpret_cast<cplx<T>*>(base + L.coef);
    U* amax = reinterpret_cast<U*>(base + L.amax);
    int* counts = reinterpret_cast<int*>(base + L.counts);
    int* offsets = reinterpret_cast<int*>(base + L.offsets);
    hipError_t e = launch_coef<T>(rho_m, w_m, K, coef, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((clear_bits_kernel<U>), dim3(1), dim3(64), 0, s, amax);
    const int64_t ab = (K + 255) / 256;
    hipLaunchKernelGGL((absmax_kernel<T>), dim3(unsigned(ab < 512 ? ab : 512)), dim3(256), 0, s, coef, K, amax);
    const T tl = T(tol);
    cplx<T>* oc = static_cast<cplx<T>*>(c_out);
    if (planar) {
        hipLaunchKernelGGL((octree_kernel<T, 2, false>), dim3(nblk), dim3(64), 0, s, coef, nm, amax, tl, max_level,
                           counts, offsets, pos, oc, level);
    } else {
        hipLaunchKernelGGL((octree_kernel<T, 3, false>), dim3(nblk), dim3(512), 0, s, coef, nm, amax, tl, max_level,
                           counts, offsets, pos, oc, level);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan(counts, offsets, nblk, base + L.temp, s);
    if (e != hipSuccess) return e;
    if (planar) {
        hipLaunchKernelGGL((octree_kernel<T, 2, true>), dim3(nblk), dim3(64), 0, s, coef, nm, amax, tl, max_level,
                           counts, offsets, pos, oc, level);
    } else {
        hipLaunchKernelGGL((octree_kernel<T, 3, true>), dim3(nblk), dim3(512), 0, s, coef, nm, amax, tl, max_level,
                           counts, offsets, pos, oc, level);
    }
    hipLaunchKernelGGL(octree_total_kernel, dim3(1), dim3(64), 0, s, counts, offsets, nblk, count_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_es_deconv(int N, int w, T* inv, hipStream_t s) {
    hipLaunchKernelGGL((es_deconv_kernel<T>), dim3(unsigned(N)), dim3(256), 0, s, N, w, inv);
    return hipGetLastError();
}

size_t nfft_workspace_bytes(int64_t m, int batch, int N, bool planar, size_t elem) {
    return nfft_ws_layout(m, batch, N, planar, elem).total;
}

size_t nfft_grid_bytes(int N, bool planar, size_t elem) {
    const int nf = 2 * N;
    const size_t full = 2 * elem * size_t(nf) * nf * (planar ? 1 : nf);
    // with the x pass fused into the line tiles only the y pass's output,
    // a quarter of the grid, lives there
    return use_lines(planar, elem) && fused_x_pass(nf) ? full / 4 : full;
}

template <typename T>
hipError_t launch_nfft_modes(const T* pos, const void* c, int64_t m, const T* R, int batch, int N, bool planar,
                             int w, const T* inv, const void* spec, void* fine, void* out, void* ws, hipStream_t s,
                             bool tiled) {
    const int nf = 2 * N;
    const bool lines = use_lines(planar, sizeof(T));
    const TileShape ts = tile_shape(nf, planar, lines);
    const NfftWs L = nfft_ws_layout(m, batch, N, planar, sizeof(T));
    char* base = static_cast<char*>(ws);
    int* counts = reinterpret_cast<int*>(base + L.counts);
    int* cursor = reinterpret_cast<int*>(base + L.cursor);
    int* offsets = reinterpret_cast<int*>(base + L.offsets);
    T* vbuf = reinterpret_cast<T*>(base + L.vbuf);
    cplx<T>* cbuf = reinterpret_cast<cplx<T>*>(base + L.cbuf);
    const int64_t nb = int64_t(ts.ntx) * ts.nty * ts.ntz * batch;
    const cplx<T>* cc = static_cast<const cplx<T>*>(c);
    cplx<T>* fg = static_cast<cplx<T>*>(fine);
    const int64_t zb = (2 * nb + 255) / 256;
        hipLaunchKernelGGL(clear_ints_kernel, dim3(unsigned(zb < 4096 ? zb : 4096)), dim3(256), 0, s, counts, nb);
    hipLaunchKernelGGL(clear_ints_kernel, dim3(unsigned(zb < 4096 ? zb : 4096)), dim3(256), 0, s, cursor, nb);
    if (m > 0) {
        const dim3 g(unsigned((m + 255) / 256), unsigned(batch));
        if (planar)
            hipLaunchKernelGGL((nfft_bin_kernel<T, 2, false>), g, dim3(256), 0, s, pos, cc, m, R, nf, w, ts, counts,
                               offsets, cursor, vbuf, cbuf);
        else
            hipLaunchKernelGGL((nfft_bin_kernel<T, 3, false>), g, dim3(256), 0, s, pos, cc, m, R, nf, w, ts, counts,
                               offsets, cursor, vbuf, cbuf);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan(counts, offsets, int(nb), base + L.temp, s);
    if (e != hipSuccess) return e;
    if (m > 0) {
        const dim3 g(unsigned((m + 255) / 256), unsigned(batch));
        if (planar)
            hipLaunchKernelGGL((nfft_bin_kernel<T, 2, true>), g, dim3(256), 0, s, pos, cc, m, R, nf, w, ts, counts,
                               offsets, cursor, vbuf, cbuf);
        else
            hipLaunchKernelGGL((nfft_bin_kernel<T, 3, true>), g, dim3(256), 0, s, pos, cc, m, R, nf, w, ts, counts,
                               offsets, cursor, vbuf, cbuf);
    }
    bool rows_done = false;
    if constexpr (std::is_same<T, float>::value) {
        if (lines && fused_x_pass(nf)) {
            e = launch_line_fft(vbuf, cbuf, counts, offsets, batch, nf, w, ts,
                                reinterpret_cast<cplx<float>*>(base + L.half), s);
            rows_done = true;
        } else if (lines) {
            switch (w) {
                case 2: launch_line_tile<2>(vbuf, cbuf, counts, offsets, batch, nf, ts, fg, s); break;
                case 3: launch_line_tile<3>(vbuf, cbuf, counts, offsets, batch, nf, ts, fg, s); break;
                case 4: launch_line_tile<4>(vbuf, cbuf, counts, offsets, batch, nf, ts, fg, s); break;
                case 5: launch_line_tile<5>(vbuf, cbuf, counts, offsets, batch, nf, ts, fg, s); break;
                case 6: launch_line_tile<6>(vbuf, cbuf, counts, offsets, batch, nf, ts, fg, s); break;
                case 7: launch_line_tile<7>(vbuf, cbuf, counts, offsets, batch, nf, ts, fg, s); break;
                case 8: launch_line_tile<8>(vbuf, cbuf, counts, offsets, batch, nf, ts, fg, s); break;
                default: return hipErrorInvalidValue;
            }
            e = hipGetLastError();
        } else {
            e = planar ? tile_width<T, 2>(vbuf, cbuf, counts, offsets, batch, nf, w, ts, fg, s)
                       : tile_width<T, 3>(vbuf, cbuf, counts, offsets, batch, nf, w, ts, fg, s);
        }
    } else {
        e = planar ? tile_width<T, 2>(vbuf, cbuf, counts, offsets, batch, nf, w, ts, fg, s)
                   : tile_width<T, 3>(vbuf, cbuf, counts, offsets, batch, nf, w, ts, fg, s);
    }
    if (e != hipSuccess) return e;
    // the y pass's output reuses the oversampled grids, free after the x pass
    return launch_pruned<T>(fg, reinterpret_cast<cplx<T>*>(base + L.half), fg, batch, N, planar, inv,
                            static_cast<const cplx<T>*>(spec), static_cast<cplx<T>*>(out), rows_done, tiled, s);
}

template hipError_t launch_octree<float>(const void*, const float*, int, bool, double, int, float*, void*, int*,
                                         int64_t*, void*, hipStream_t);
template hipError_t launch_octree<double>(const void*, const double*, int, bool, double, int, double*, void*, int*,
                                          int64_t*, void*, hipStream_t);
template hipError_t launch_es_deconv<float>(int, int, float*, hipStream_t);
template hipError_t launch_es_deconv<double>(int, int, double*, hipStream_t);
template hipError_t launch_nfft_modes<float>(const float*, const void*, int64_t, const float*, int, int, bool, int,
                                             const float*, const void*, void*, void*, void*, hipStream_t, bool);
template hipError_t launch_nfft_modes<double>(const double*, const void*, int64_t, const double*, int, int, bool,
                                              int, const double*, const void*, void*, void*, void*, hipStream_t,
                                              bool);

}  // namespace sdf
