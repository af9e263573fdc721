// Exclusive prefix sums and a stable key-value radix sort (gfx950).
//
// The scan is hierarchical: blocks of 256 threads scan 2048 values each
// (eight per thread, then the thread totals across the block), one block
// scans the block totals, and a third pass adds each block's offset.
//
// The sort is least-significant-digit first with 8-bit digits.  Per pass:
//   count    each block takes a tile of kSortTile keys and counts its digits
//            (LDS atomics) into counts[digit][block];
//   scan     an exclusive scan of counts in digit-major order gives every
//            (digit, block) its first output position;
//   scatter  each block walks its tile in order, 256 keys per round: inside
//            a wave the lanes with the same digit are found from one ballot
//            per digit bit, and a lane's rank is the number of such lanes
//            below it; the waves of a round are ordered by a per-digit
//            count in LDS, and a running per-digit count carries the order
//            across rounds.  Equal keys therefore keep their input order.
#include <utility>

#include "common.hpp"
#include "launch.hpp"

namespace sdf {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanBlock * kScanPer;  // values per block
constexpr int kSortBlock = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortBlock * kSortRounds;  // keys per block
constexpr int kDigits = 256;
static_assert(kScanBlock == 4 * 64, "block_exclusive sums the totals of four waves");

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// exclusive scan of the block's kScanBlock thread totals in LDS; returns the
// thread's offset and writes the block total to *total
__device__ __forceinline__ int block_exclusive(int v, int* __restrict__ sh, int* total) {
    const int t = int(threadIdx.x), lane = t & 63, wave = t >> 6;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; ++w) base += sh[w];
    *total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return base + incl - v;
}

__global__ __launch_bounds__(kScanBlock) void scan_tiles_kernel(const int* __restrict__ in, int* __restrict__ out,
                                                                int64_t n, int* __restrict__ sums) {
    __shared__ int sh[kScanBlock / 64];
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanPer;
    int v[kScanPer];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_exclusive(s, sh, &total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// one block: exclusive scan of the nb block totals in place, kScanTile at a time
__global__ __launch_bounds__(kScanBlock) void scan_sums_kernel(int* __restrict__ sums, int64_t nb) {
    __shared__ int sh[kScanBlock / 64];
    int carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanTile) {
        const int64_t base = b0 + int64_t(threadIdx.x) * kScanPer;
        int v[kScanPer];
        int s = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = base + k < nb ? sums[base + k] : 0;
            s += v[k];
        }
        int total;
        int run = carry + block_exclusive(s, sh, &total);
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if (base + k < nb) sums[base + k] = run;
            run += v[k];
        }
        carry += total;
    }
}

__global__ __launch_bounds__(kScanBlock) void scan_add_kernel(int* __restrict__ out, int64_t n,
                                                              const int* __restrict__ sums) {
    const int add = sums[blockIdx.x];
    if (blockIdx.x == 0) return;
    const int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + int64_t(k) * kScanBlock;
        if (i < n) out[i] += add;
    }
}

__global__ __launch_bounds__(kSortBlock) void sort_count_kernel(const unsigned* __restrict__ keys, int64_t n,
                                                                int shift, int nblocks, int* __restrict__ counts) {
    __shared__ int hist[kDigits];
    for (int d = int(threadIdx.x); d < kDigits; d += kSortBlock) hist[d] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + int64_t(r) * kSortBlock + threadIdx.x;
        if (i < n) atomicAdd(&hist[(keys[i] >> shift) & (kDigits - 1)], 1);
    }
    __syncthreads();
    for (int d = int(threadIdx.x); d < kDigits; d += kSortBlock)
        counts[int64_t(d) * nblocks + blockIdx.x] = hist[d];
}

__global__ __launch_bounds__(kSortBlock) void sort_scatter_kernel(const unsigned* __restrict__ keys_in,
                                                                  const int* __restrict__ vals_in, int64_t n,
                                                                  int shift, int nblocks,
                                                                  const int* __restrict__ offsets,
                                                                  unsigned* __restrict__ keys_out,
                                                                  int* __restrict__ vals_out) {
    constexpr int W = kSortBlock / 64;
    __shared__ int start[kDigits];    // first output position of each digit in this block
    __shared__ int wcount[W][kDigits];  // keys of each digit per wave in the current round
    for (int d = int(threadIdx.x); d < kDigits; d += kSortBlock) {
        start[d] = offsets[int64_t(d) * nblocks + blockIdx.x];
        for (int w = 0; w < W; ++w) wcount[w][d] = 0;
    }
    __syncthreads();
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
    const uint64_t below = (uint64_t(1) << lane) - 1;
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + int64_t(r) * kSortBlock + threadIdx.x;
        const bool live = i < n;
        const unsigned key = live ? keys_in[i] : 0u;
        const int val = live ? vals_in[i] : 0;
        const int d = int((key >> shift) & (kDigits - 1));
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(live);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        const int rank = __popcll(peers & below);
        if (live && rank == 0) wcount[wave][d] = __popcll(peers);
        __syncthreads();
        if (live) {
            int pos = start[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcount[w][d];
            if (pos >= 0 && pos < n) {
                keys_out[pos] = key;
                vals_out[pos] = val;
            }
        }
        __syncthreads();
        for (int dd = int(threadIdx.x); dd < kDigits; dd += kSortBlock) {
            int s = 0;
            for (int w = 0; w < W; ++w) {
                s += wcount[w][dd];
                wcount[w][dd] = 0;
            }
            start[dd] += s;
        }
        __syncthreads();
    }
}

}  // namespace

size_t scan_temp_bytes(int64_t n) { return al256(sizeof(int) * size_t((n + kScanTile - 1) / kScanTile + 1)); }

hipError_t launch_exclusive_scan(const int* in, int* out, int64_t n, void* temp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int* sums = static_cast<int*>(temp);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(unsigned(nb)), dim3(kScanBlock), 0, s, in, out, n, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, s, sums, nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3(unsigned(nb)), dim3(kScanBlock), 0, s, out, n, sums);
    return hipGetLastError();
}

size_t sort_temp_bytes(int64_t n) {
    const int64_t nblocks = (n + kSortTile - 1) / kSortTile;
    const int64_t m = int64_t(kDigits) * nblocks;
    return 2 * al256(sizeof(int) * size_t(m)) + scan_temp_bytes(m);
}

hipError_t launch_sort_pairs(unsigned* keys, int* vals, unsigned* keys_alt, int* vals_alt, int64_t n, int bits,
                             void* temp, hipStream_t s, unsigned** keys_sorted, int** vals_sorted) {
    *keys_sorted = keys;
    *vals_sorted = vals;
    if (n <= 0) return hipSuccess;
    const int64_t nblocks = (n + kSortTile - 1) / kSortTile;
    const int64_t m = int64_t(kDigits) * nblocks;
    char* t = static_cast<char*>(temp);
    int* counts = reinterpret_cast<int*>(t);
    int* offsets = reinterpret_cast<int*>(t + al256(sizeof(int) * size_t(m)));
    void* scan_tmp = t + 2 * al256(sizeof(int) * size_t(m));
    unsigned *ki = keys, *ko = keys_alt;
    int *vi = vals, *vo = vals_alt;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(sort_count_kernel, dim3(unsigned(nblocks)), dim3(kSortBlock), 0, s, ki, n, shift,
                           int(nblocks), counts);
        hipError_t e = launch_exclusive_scan(counts, offsets, m, scan_tmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(sort_scatter_kernel, dim3(unsigned(nblocks)), dim3(kSortBlock), 0, s, ki, vi, n, shift,
                           int(nblocks), offsets, ko, vo);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    *keys_sorted = ki;
    *vals_sorted = vi;
    return hipGetLastError();
}

}  // namespace sdf
