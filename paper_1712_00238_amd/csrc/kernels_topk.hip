// Top-k rotations by score (descending, ties by lower index): bitonic sort
// of (score, index) pairs padded to a power of two.  Small inputs sort in one
// block in LDS; larger inputs use one launch per compare-exchange stage.
#include <climits>

#include "common.hpp"
#include "launch.hpp"

namespace sdf {

namespace {

template <typename T>
__device__ __forceinline__ bool before(T a, int ia, T b, int ib) {  // a ranks before b
    return a > b || (a == b && ia < ib);
}

template <typename T>
__global__ void topk_init_kernel(const T* __restrict__ s, int64_t n, int64_t P, T* __restrict__ v,
                                 int* __restrict__ id) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= P) return;
    if (i < n) {
        T x = s[i];
        v[i] = (x == x) ? x : T(-INFINITY);
        id[i] = int(i);
    } else {
        v[i] = T(-INFINITY);
        id[i] = INT_MAX;
    }
}

template <typename T>
__global__ void bitonic_stage_kernel(T* __restrict__ v, int* __restrict__ id, int64_t P, int64_t k, int64_t j) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const bool up = (i & k) == 0;  // this subsequence sorts in ranking order
    const T a = v[i], b = v[l];
    const int ia = id[i], ib = id[l];
    const bool swap = up ? before(b, ib, a, ia) : before(a, ia, b, ib);
    if (swap) {
        v[i] = b;
        v[l] = a;
        id[i] = ib;
        id[l] = ia;
    }
}

constexpr int kLdsSort = 2048;

template <typename T>
__global__ __launch_bounds__(1024) void bitonic_lds_kernel(T* __restrict__ v, int* __restrict__ id, int P) {
    __shared__ T sv[kLdsSort];
    __shared__ int si[kLdsSort];
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        sv[i] = v[i];
        si[i] = id[i];
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const T a = sv[i], b = sv[l];
                    const int ia = si[i], ib = si[l];
                    const bool swap = up ? before(b, ib, a, ia) : before(a, ia, b, ib);
                    if (swap) {
                        sv[i] = b;
                        sv[l] = a;
                        si[i] = ib;
                        si[l] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        v[i] = sv[i];
        id[i] = si[i];
    }
}

__global__ void topk_copy_kernel(const int* __restrict__ id, int64_t k, int32_t* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < k) out[i] = id[i];
}

int64_t pow2_at_least(int64_t n) {
    int64_t p = 2;
    while (p < n) p <<= 1;
    return p;
}

}  // namespace

size_t topk_workspace_bytes(int64_t n) {
    const int64_t P = pow2_at_least(n);
    return size_t(P) * (sizeof(double) + sizeof(int)) + 512;
}

template <typename T>
hipError_t launch_topk(const T* scores, int64_t n, int64_t k, void* ws, int32_t* idx_out, hipStream_t s) {
    const int64_t P = pow2_at_least(n);
    T* v = static_cast<T*>(ws);
    int* id = reinterpret_cast<int*>(static_cast<char*>(ws) + ((size_t(P) * sizeof(T) + 255) / 256 * 256));
    const unsigned g = unsigned((P + 255) / 256);
    hipLaunchKernelGGL(topk_init_kernel<T>, dim3(g), dim3(256), 0, s, scores, n, P, v, id);
    if (P <= kLdsSort) {
        hipLaunchKernelGGL(bitonic_lds_kernel<T>, dim3(1), dim3(1024), 0, s, v, id, int(P));
    } else {
        for (int64_t kk = 2; kk <= P; kk <<= 1)
            for (int64_t j = kk >> 1; j > 0; j >>= 1)
                hipLaunchKernelGGL(bitonic_stage_kernel<T>, dim3(g), dim3(256), 0, s, v, id, P, kk, j);
    }
    hipLaunchKernelGGL(topk_copy_kernel, dim3(unsigned((k + 255) / 256)), dim3(256), 0, s, id, k, idx_out);
    return hipGetLastError();
}

template hipError_t launch_topk<float>(const float*, int64_t, int64_t, void*, int32_t*, hipStream_t);
template hipError_t launch_topk<double>(const double*, int64_t, int64_t, void*, int32_t*, hipStream_t);

}  // namespace sdf
