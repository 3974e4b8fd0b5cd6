// FP64 inner product for the adjoint (dot-product) check and for losses.
// Deterministic: a fixed grid writes one partial per block through a fixed
// reduction tree; a second single-block kernel sums the partials in fixed order.
#include "radon_common.hpp"
#include "radon_launch.hpp"

namespace radon {

constexpr int kDotThreads = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int w = kDotThreads / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    return sh[0];
}

template <typename T>
__global__ __launch_bounds__(kDotThreads) void dot_partial(const T *__restrict__ a,
                                                           const T *__restrict__ b, long long n,
                                                           double *__restrict__ partials) {
    __shared__ double sh[kDotThreads];
    double s = 0.0;
    const long long stride = (long long)gridDim.x * kDotThreads;
    for (long long j = (long long)blockIdx.x * kDotThreads + threadIdx.x; j < n; j += stride)
        s = fma((double)Store<T>::load(a + j), (double)Store<T>::load(b + j), s);
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kDotThreads) void dot_final(const double *__restrict__ partials,
                                                         int np, double *__restrict__ out) {
    __shared__ double sh[kDotThreads];
    double s = 0.0;
    for (int j = threadIdx.x; j < np; j += kDotThreads) s += partials[j];
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) *out = tot;
}

template <typename T>
static hipError_t launch_dot(const void *a, const void *b, long long n, double *out,
                             double *partials, int np, hipStream_t s) {
    hipLaunchKernelGGL(dot_partial<T>, dim3(np), dim3(kDotThreads), 0, s, (const T *)a,
                       (const T *)b, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dot_final, dim3(1), dim3(kDotThreads), 0, s, partials, np, out);
    return hipGetLastError();
}

hipError_t launch_dot_f64(const void *a, const void *b, long long n, int dtype, double *out,
                          double *partials, int n_partials, hipStream_t s) {
    switch (dtype) {
    case F32: return launch_dot<float>(a, b, n, out, partials, n_partials, s);
    case F16: return launch_dot<__half>(a, b, n, out, partials, n_partials, s);
    case BF16: return launch_dot<bf16_t>(a, b, n, out, partials, n_partials, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
