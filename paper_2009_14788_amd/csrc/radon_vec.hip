// Vector steps of the iterative solvers (TorchRadon Sec. 4.2-4.3): per-system FP64
// inner products and the scaled update out = u + c v whose coefficient c is a ratio of
// two such inner products read from device memory, so a conjugate-gradient iteration
// never waits on the host.  A batch holds `batch` independent systems of n elements
// each, stored one after another.
//
// Inner products are deterministic: system b is cut into `chunks` contiguous pieces,
// each block reduces one piece through a fixed tree into partials[b * chunks + c], and
// one block per system sums its partials in a fixed order.
#include <map>
#include <mutex>

#include "radon_common.hpp"
#include "radon_launch.hpp"

namespace radon {

constexpr int kVecThreads = 256;

__device__ __forceinline__ double tree_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int w = kVecThreads / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    return sh[0];
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void dot_rows_partial(const T *__restrict__ a,
                                                                const T *__restrict__ b,
                                                                long long n, long long piece,
                                                                double *__restrict__ partials) {
    __shared__ double sh[kVecThreads];
    const long long base = (long long)blockIdx.y * n;
    const long long lo = (long long)blockIdx.x * piece;
    const long long hi = lo + piece < n ? lo + piece : n;
    double s = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += kVecThreads)
        s = fma((double)Store<T>::load(a + base + i), (double)Store<T>::load(b + base + i), s);
    const double tot = tree_sum(s, sh);
    if (threadIdx.x == 0) partials[(long long)blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

__global__ __launch_bounds__(kVecThreads) void dot_rows_final(const double *__restrict__ partials,
                                                              int chunks, double *__restrict__ out) {
    __shared__ double sh[kVecThreads];
    double s = 0.0;
    for (int j = threadIdx.x; j < chunks; j += kVecThreads)
        s += partials[(long long)blockIdx.x * chunks + j];
    const double tot = tree_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

// c_b = c0 * num[b] / den[b] (a missing array reads as 1; 0 when den[b] == 0); where
// c_b == 0 the output is u exactly and v is not read.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void axpy_ratio_rows(const T *__restrict__ u,
                                                               const T *__restrict__ v,
                                                               T *__restrict__ out,
                                                               const double *__restrict__ num,
                                                               const double *__restrict__ den,
                                                               double c0, long long n) {
    const int b = blockIdx.y;
    double c = c0;
    if (num) c *= num[b];
    if (den) c = den[b] == 0.0 ? 0.0 : c / den[b];
    const long long base = (long long)b * n;
    const long long stride = (long long)gridDim.x * kVecThreads;
    if (c == 0.0) {
        if (out != u)
            for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride)
                out[base + i] = u[base + i];
        return;
    }
    for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        const double r = fma(c, (double)Store<T>::load(v + base + i), (double)Store<T>::load(u + base + i));
        Store<T>::store(out + base + i, (float)r);
    }
}

// A reproducible pseudo-random pattern in [-0.5, 0.5) (an integer hash of the index
// and seed), for buffers whose content only has to look like data.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void fill_pattern(T *__restrict__ p, long long n,
                                                            unsigned seed) {
    const long long stride = (long long)gridDim.x * kVecThreads;
    for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        unsigned h = (unsigned)i * 2654435761u ^ (unsigned)(i >> 32) ^ seed;
        h ^= h >> 15;
        h *= 0x2c1b3c6du;
        h ^= h >> 12;
        h *= 0x297a2d39u;
        h ^= h >> 15;
        Store<T>::store(p + i, (float)(h >> 8) * (1.0f / 16777216.0f) - 0.5f);
    }
}

hipError_t launch_fill_pattern(void *p, long long n, int dtype, unsigned seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + kVecThreads - 1) / kVecThreads;
    if (blocks > 4096) blocks = 4096;
    switch (dtype) {
    case F32:
        hipLaunchKernelGGL(fill_pattern<float>, dim3((unsigned)blocks), dim3(kVecThreads), 0, s,
                           (float *)p, n, seed);
        break;
    case F16:
        hipLaunchKernelGGL(fill_pattern<__half>, dim3((unsigned)blocks), dim3(kVecThreads), 0, s,
                           (__half *)p, n, seed);
        break;
    case BF16:
        hipLaunchKernelGGL(fill_pattern<bf16_t>, dim3((unsigned)blocks), dim3(kVecThreads), 0, s,
                           (bf16_t *)p, n, seed);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int dot_rows_chunks(long long n) {
    const long long per = (long long)kVecThreads * 16;
    long long c = (n + per - 1) / per;
    return (int)(c < 1 ? 1 : c > kDotRowChunks ? kDotRowChunks : c);
}

template <typename T>
static hipError_t dot_rows_typed(const void *a, const void *b, long long n, int batch, double *out,
                                 double *partials, hipStream_t s) {
    const int chunks = dot_rows_chunks(n);
    const long long piece = (n + chunks - 1) / chunks;
    hipLaunchKernelGGL(dot_rows_partial<T>, dim3(chunks, batch), dim3(kVecThreads), 0, s,
                       (const T *)a, (const T *)b, n, piece, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dot_rows_final, dim3(batch), dim3(kVecThreads), 0, s,
                       (const double *)partials, chunks, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fixed scratch
// Partials of the no-allocation inner products: one array per GPU, part of the code
// object, so it exists from module load until the process ends.  In host code the
// name `scratch` is only a stand-in for the symbol; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) double scratch[kStaticDotPartials];

static std::mutex g_static_mutex;
static std::map<int, double *> g_static_ptr;   // device -> address of its `scratch`

hipError_t static_dot_partials(double **out) {
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_static_mutex);
    auto it = g_static_ptr.find(device);
    if (it == g_static_ptr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        it = g_static_ptr.emplace(device, static_cast<double *>(p)).first;
    }
    *out = it->second;
    return hipSuccess;
}

hipError_t launch_dot_rows(const void *a, const void *b, long long n, int batch, int dtype,
                           double *out, double *partials, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    if (n <= 0) {
        // empty systems: every inner product is 0 (the final pass reads zero partials)
        hipLaunchKernelGGL(dot_rows_final, dim3(batch), dim3(kVecThreads), 0, s,
                           (const double *)partials, 0, out);
        return hipGetLastError();
    }
    switch (dtype) {
    case F32: return dot_rows_typed<float>(a, b, n, batch, out, partials, s);
    case F16: return dot_rows_typed<__half>(a, b, n, batch, out, partials, s);
    case BF16: return dot_rows_typed<bf16_t>(a, b, n, batch, out, partials, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t axpy_typed(const void *u, const void *v, void *out, const double *num,
                             const double *den, double c0, long long n, int batch, hipStream_t s) {
    long long blocks = (n + kVecThreads * 4 - 1) / (kVecThreads * 4);
    const long long cap = batch >= 256 ? 4 : 1024 / batch + 1;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(axpy_ratio_rows<T>, dim3((unsigned)blocks, batch), dim3(kVecThreads), 0, s,
                       (const T *)u, (const T *)v, (T *)out, num, den, c0, n);
    return hipGetLastError();
}

hipError_t launch_axpy_ratio(const void *u, const void *v, void *out, const double *num,
                             const double *den, double c0, long long n, int batch, int dtype,
                             hipStream_t s) {
    if (batch <= 0 || n <= 0) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    switch (dtype) {
    case F32: return axpy_typed<float>(u, v, out, num, den, c0, n, batch, s);
    case F16: return axpy_typed<__half>(u, v, out, num, den, c0, n, batch, s);
    case BF16: return axpy_typed<bf16_t>(u, v, out, num, den, c0, n, batch, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
