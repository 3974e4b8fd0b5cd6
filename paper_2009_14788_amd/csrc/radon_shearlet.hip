// Alpha-shearlet transform on the GPU (TorchRadon Sec. 2.1 lists it, Sec. 3.2
// compares it with AlphaTransforms): the Fourier filters psi_m of a Parseval
// alpha-shearlet system are built once on the host; every transform is then FFTs and
// products in the frequency domain, for a batch of images at once.
//
// Both directions exploit that every psi_m is real and even (so each channel's
// coefficients are real): channels 2p and 2p + 1 travel as the real and imaginary
// parts of one complex field.
//
//   forward  c_m = Re IFFT2(FFT2(x) psi_m):
//     1. row FFTs of the images                      -> X1 [C][H][W]
//     2. per tile of TC columns: column FFTs (= FFT2(x) on those columns), then per
//        pair p: times psi_2p + i psi_2p+1, inverse column FFTs -> Y [C][P][H][W]
//     3. per row of Y: inverse row FFT; real part -> channel 2p, imaginary -> 2p + 1
//   adjoint  x = Re IFFT2(sum_m FFT2(c_m) psi_m) = Re IFFT2(sum_p (psi_2p - i psi_2p+1)
//            FFT2(c_2p + i c_2p+1)):
//     1. per row of every pair: row FFT of c_2p + i c_2p+1  -> U [C][P][H][W]
//     2. per tile of TC columns and group of pairs: column FFTs, times
//        psi_2p - i psi_2p+1, summed over the group's pairs, inverse column FFTs
//                                                     -> V [G][C][H][W]
//     3. per image row: sum of the G partials, inverse row FFT, real part -> x
//
// Transforms are the radix-4/8 Stockham FFTs of radon_fft.hpp in LDS; inverse
// transforms conjugate in and out; the 1/(H W) of the inverse is applied once, at the
// output.  Column tiles are stored one column per LDS sequence with a one-element pad,
// so the row-order loads and stores of a tile spread over the banks.  FP32 arithmetic
// for every storage type.
#include <algorithm>

#include "radon_common.hpp"
#include "radon_fft.hpp"
#include "radon_shearlet.hpp"

namespace radon {

constexpr int kShThreads = 256;

// rows per block of the row kernels: NR * W = max(2048, W) complex values in LDS
__host__ __device__ constexpr int sh_rows_per_block(int log2w) {
    return log2w >= 11 ? 1 : (2048 >> log2w);
}
// columns per block of the column kernels: TC * H <= 4096 (two padded buffers, <= 66 KB)
__host__ __device__ constexpr int sh_log2_tile(int log2h) {
    return log2h >= 12 ? 0 : (12 - log2h > 3 ? 3 : 12 - log2h);
}

// 1a. forward row FFTs of real images: X1[g] = FFT(x[g]) for rows g < rows
template <typename T, int LOG2W>
__global__ __launch_bounds__(kShThreads) void sh_rows_image(const T *__restrict__ x, float2 *__restrict__ X1,
                                                            long long rows, const float2 *__restrict__ tw) {
    constexpr int W = 1 << LOG2W, NR = sh_rows_per_block(LOG2W);
    extern __shared__ float2 buf[];
    const long long g0 = (long long)blockIdx.x * NR;
    for (int i = threadIdx.x; i < NR * W; i += kShThreads) {
        const long long g = g0 + (i >> LOG2W);
        buf[i] = make_float2(g < rows ? Store<T>::load(x + g * W + (i & (W - 1))) : 0.0f, 0.0f);
    }
    __syncthreads();
    fft_multi<kShThreads, NR, W, LOG2W>(buf, tw);
    for (int i = threadIdx.x; i < NR * W; i += kShThreads) {
        const long long g = g0 + (i >> LOG2W);
        if (g < rows) X1[g * W + (i & (W - 1))] = buf[i];
    }
}

// 1b. forward row FFTs of channel pairs: U[g] = FFT(c_2p[r] + i c_2p+1[r]), row
// g = (ci P + p) H + r
template <typename T, int LOG2W>
__global__ __launch_bounds__(kShThreads) void sh_rows_coeffs(const T *__restrict__ c, float2 *__restrict__ U,
                                                             long long rows, int log2h, int pairs,
                                                             int channels, const float2 *__restrict__ tw) {
    constexpr int W = 1 << LOG2W, NR = sh_rows_per_block(LOG2W);
    extern __shared__ float2 buf[];
    const long long g0 = (long long)blockIdx.x * NR;
    const long long H = 1ll << log2h;
    for (int i = threadIdx.x; i < NR * W; i += kShThreads) {
        const long long g = g0 + (i >> LOG2W);
        float2 v = make_float2(0.0f, 0.0f);
        if (g < rows) {
            const long long r = g & (H - 1), q = g >> log2h;
            const long long ci = q / pairs, m = 2 * (q - ci * pairs);
            const long long k = i & (W - 1);
            v.x = Store<T>::load(c + ((ci * channels + m) * H + r) * W + k);
            if (m + 1 < channels) v.y = Store<T>::load(c + ((ci * channels + m + 1) * H + r) * W + k);
        }
        buf[i] = v;
    }
    __syncthreads();
    fft_multi<kShThreads, NR, W, LOG2W>(buf, tw);
    for (int i = threadIdx.x; i < NR * W; i += kShThreads) {
        const long long g = g0 + (i >> LOG2W);
        if (g < rows) U[g * W + (i & (W - 1))] = buf[i];
    }
}

// 2a. forward column pass (grid: W / TC column tiles x pair groups x images)
template <int LOG2H>
__global__ __launch_bounds__(kShThreads) void sh_cols_forward(const float2 *__restrict__ X1,
                                                              const float2 *__restrict__ psi,
                                                              float2 *__restrict__ Y, int log2w, int pairs,
                                                              int per_group, const float2 *__restrict__ tw) {
    constexpr int H = 1 << LOG2H, LOG2TC = sh_log2_tile(LOG2H), TC = 1 << LOG2TC, STRIDE = H + 1;
    extern __shared__ float2 lds[];
    float2 *Xs = lds, *Ws = lds + TC * STRIDE;
    const long long W = 1ll << log2w;
    const int col0 = blockIdx.x * TC;
    const int p0 = blockIdx.y * per_group, p1 = min(pairs, p0 + per_group);
    const long long ci = blockIdx.z;
    const float2 *src = X1 + ci * H * W + col0;
    for (int i = threadIdx.x; i < TC * H; i += kShThreads)
        Xs[(i & (TC - 1)) * STRIDE + (i >> LOG2TC)] = src[(long long)(i >> LOG2TC) * W + (i & (TC - 1))];
    __syncthreads();
    fft_multi<kShThreads, TC, STRIDE, LOG2H>(Xs, tw);
    for (int p = p0; p < p1; ++p) {
        const float2 *f = psi + ((long long)p * W + col0) * H;
        for (int i = threadIdx.x; i < TC * H; i += kShThreads) {
            const int j = i >> LOG2H, k = i & (H - 1);
            const float2 a = Xs[j * STRIDE + k], h = f[i];
            // conj(a (h.x + i h.y)): the inverse transform runs on the conjugate
            Ws[j * STRIDE + k] = make_float2(a.x * h.x - a.y * h.y, -(a.x * h.y + a.y * h.x));
        }
        __syncthreads();
        fft_multi<kShThreads, TC, STRIDE, LOG2H>(Ws, tw);
        float2 *dst = Y + (ci * pairs + p) * H * W + col0;
        for (int i = threadIdx.x; i < TC * H; i += kShThreads) {
            const float2 v = Ws[(i & (TC - 1)) * STRIDE + (i >> LOG2TC)];
            dst[(long long)(i >> LOG2TC) * W + (i & (TC - 1))] = cconj(v);
        }
        __syncthreads();
    }
}

// 2b. adjoint column pass (grid: W / TC column tiles x pair groups x images): the
// group's partial sum over its pairs, back to rows in the spatial domain
template <int LOG2H>
__global__ __launch_bounds__(kShThreads) void sh_cols_adjoint(const float2 *__restrict__ U,
                                                              const float2 *__restrict__ psi,
                                                              float2 *__restrict__ V, int log2w, int pairs,
                                                              int per_group, int chunk,
                                                              const float2 *__restrict__ tw) {
    constexpr int H = 1 << LOG2H, LOG2TC = sh_log2_tile(LOG2H), TC = 1 << LOG2TC, STRIDE = H + 1;
    extern __shared__ float2 lds[];
    float2 *Us = lds, *As = lds + TC * STRIDE;
    const long long W = 1ll << log2w;
    const int col0 = blockIdx.x * TC;
    const int p0 = blockIdx.y * per_group, p1 = min(pairs, p0 + per_group);
    const long long ci = blockIdx.z;
    for (int i = threadIdx.x; i < TC * H; i += kShThreads)
        As[(i >> LOG2H) * STRIDE + (i & (H - 1))] = make_float2(0.0f, 0.0f);
    for (int p = p0; p < p1; ++p) {
        const float2 *src = U + (ci * pairs + p) * H * W + col0;
        for (int i = threadIdx.x; i < TC * H; i += kShThreads)
            Us[(i & (TC - 1)) * STRIDE + (i >> LOG2TC)] = src[(long long)(i >> LOG2TC) * W + (i & (TC - 1))];
        __syncthreads();
        fft_multi<kShThreads, TC, STRIDE, LOG2H>(Us, tw);
        const float2 *f = psi + ((long long)p * W + col0) * H;
        for (int i = threadIdx.x; i < TC * H; i += kShThreads) {
            const int e = (i >> LOG2H) * STRIDE + (i & (H - 1));
            const float2 a = Us[e], h = f[i];
            float2 acc = As[e];
            // a (h.x - i h.y)
            acc.x += a.x * h.x + a.y * h.y;
            acc.y += a.y * h.x - a.x * h.y;
            As[e] = acc;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < TC * H; i += kShThreads) {
        const int e = (i >> LOG2H) * STRIDE + (i & (H - 1));
        As[e] = cconj(As[e]);
    }
    __syncthreads();
    fft_multi<kShThreads, TC, STRIDE, LOG2H>(As, tw);
    float2 *dst = V + ((long long)blockIdx.y * chunk + ci) * H * W + col0;
    for (int i = threadIdx.x; i < TC * H; i += kShThreads) {
        const float2 v = As[(i & (TC - 1)) * STRIDE + (i >> LOG2TC)];
        dst[(long long)(i >> LOG2TC) * W + (i & (TC - 1))] = cconj(v);
    }
}

// 3a. forward output: inverse row FFT of Y's rows, real part to channel 2p and
// imaginary part to channel 2p + 1 (row g = (ci P + p) H + r)
template <typename T, int LOG2W>
__global__ __launch_bounds__(kShThreads) void sh_rows_to_coeffs(const float2 *__restrict__ Y, T *__restrict__ c,
                                                                long long rows, int log2h, int pairs,
                                                                int channels, float inv,
                                                                const float2 *__restrict__ tw) {
    constexpr int W = 1 << LOG2W, NR = sh_rows_per_block(LOG2W);
    extern __shared__ float2 buf[];
    const long long g0 = (long long)blockIdx.x * NR;
    const long long H = 1ll << log2h;
    for (int i = threadIdx.x; i < NR * W; i += kShThreads) {
        const long long g = g0 + (i >> LOG2W);
        buf[i] = g < rows ? cconj(Y[g * W + (i & (W - 1))]) : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
    fft_multi<kShThreads, NR, W, LOG2W>(buf, tw);
    for (int i = threadIdx.x; i < NR * W; i += kShThreads) {
        const long long g = g0 + (i >> LOG2W);
        if (g >= rows) continue;
        const long long r = g & (H - 1), q = g >> log2h;
        const long long ci = q / pairs, m = 2 * (q - ci * pairs);
        const long long k = i & (W - 1);
        const float2 v = buf[i];        // conj of the inverse transform
        Store<T>::store(c + ((ci * channels + m) * H + r) * W + k, v.x * inv);
        if (m + 1 < channels) Store<T>::store(c + ((ci * channels + m + 1) * H + r) * W + k, -v.y * inv);
    }
}

// 3b. adjoint output: x[g] = Re IFFT(sum over the G partials of V), image row g
template <typename T, int LOG2W>
__global__ __launch_bounds__(kShThreads) void sh_rows_to_image(const float2 *__restrict__ V, T *__restrict__ x,
                                                               long long rows, int groups, float inv,
                                                               const float2 *__restrict__ tw) {
    constexpr int W = 1 << LOG2W, NR = sh_rows_per_block(LOG2W);
    extern __shared__ float2 buf[];
    const long long g0 = (long long)blockIdx.x * NR;
    const long long plane = rows * W;
    for (int i = threadIdx.x; i < NR * W; i += kShThreads) {
        const long long g = g0 + (i >> LOG2W);
        float2 v = make_float2(0.0f, 0.0f);
        if (g < rows) {
            const float2 *src = V + g * W + (i & (W - 1));
            for (int q = 0; q < groups; ++q) v = cadd(v, src[q * plane]);
        }
        buf[i] = cconj(v);
    }
    __syncthreads();
    fft_multi<kShThreads, NR, W, LOG2W>(buf, tw);
    for (int i = threadIdx.x; i < NR * W; i += kShThreads) {
        const long long g = g0 + (i >> LOG2W);
        if (g < rows) Store<T>::store(x + g * W + (i & (W - 1)), buf[i].x * inv);
    }
}

// ---------------------------------------------------------------- host side
static int groups_for(const ShearletDims &d, int chunk, int max_groups) {
    const int tiles = 1 << (d.log2w - sh_log2_tile(d.log2h));
    const int want = std::max(1, 2048 / std::max(1, chunk * tiles));
    return std::min({want, d.pairs, max_groups});
}

static int per_group(int pairs, int groups) { return (pairs + groups - 1) / groups; }

int shearlet_chunk(const ShearletDims &d, int batch) {
    const size_t field = (size_t)d.pairs << (d.log2w + d.log2h);          // complex values per image
    const size_t cap = ((size_t)512 << 20) / (field * sizeof(float2));
    return (int)std::max<size_t>(1, std::min<size_t>(cap, (size_t)std::max(batch, 1)));
}

size_t shearlet_workspace_bytes(const ShearletDims &d, int chunk, bool adjoint) {
    const size_t plane = (size_t)1 << (d.log2w + d.log2h);
    const size_t fields = (size_t)chunk * d.pairs * plane;
    if (!adjoint) return (fields + (size_t)chunk * plane) * sizeof(float2);
    const int g = per_group(d.pairs, groups_for(d, chunk, 8));
    const int groups = (d.pairs + g - 1) / g;
    return (fields + (size_t)groups * chunk * plane) * sizeof(float2);
}

template <typename T, int LOG2W>
static hipError_t launch_rows(bool adjoint, int stage, const ShearletDims &d, const float2 *tw_w,
                              const void *src, void *dst, long long rows, int groups, float inv,
                              hipStream_t s) {
    constexpr int NR = sh_rows_per_block(LOG2W);
    const size_t lds = (size_t)NR * sizeof(float2) << LOG2W;
    const dim3 grid((unsigned)((rows + NR - 1) / NR)), block(kShThreads);
    if (!adjoint && stage == 0)
        hipLaunchKernelGGL((sh_rows_image<T, LOG2W>), grid, block, lds, s, (const T *)src, (float2 *)dst,
                           rows, tw_w);
    else if (!adjoint)
        hipLaunchKernelGGL((sh_rows_to_coeffs<T, LOG2W>), grid, block, lds, s, (const float2 *)src,
                           (T *)dst, rows, d.log2h, d.pairs, d.channels, inv, tw_w);
    else if (stage == 0)
        hipLaunchKernelGGL((sh_rows_coeffs<T, LOG2W>), grid, block, lds, s, (const T *)src, (float2 *)dst,
                           rows, d.log2h, d.pairs, d.channels, tw_w);
    else
        hipLaunchKernelGGL((sh_rows_to_image<T, LOG2W>), grid, block, lds, s, (const float2 *)src,
                           (T *)dst, rows, groups, inv, tw_w);
    return hipGetLastError();
}

template <typename T>
static hipError_t rows_dispatch(bool adjoint, int stage, const ShearletDims &d, const float2 *tw_w,
                                const void *src, void *dst, long long rows, int groups, float inv,
                                hipStream_t s) {
    switch (d.log2w) {
#define RADON_SH_ROWS(M) \
    case M: return launch_rows<T, M>(adjoint, stage, d, tw_w, src, dst, rows, groups, inv, s);
    RADON_SH_ROWS(4) RADON_SH_ROWS(5) RADON_SH_ROWS(6) RADON_SH_ROWS(7) RADON_SH_ROWS(8)
    RADON_SH_ROWS(9) RADON_SH_ROWS(10) RADON_SH_ROWS(11) RADON_SH_ROWS(12)
#undef RADON_SH_ROWS
    default: return hipErrorInvalidValue;
    }
}

template <int LOG2H>
static hipError_t launch_cols(bool adjoint, const ShearletDims &d, const float2 *psi, const float2 *tw_h,
                              const float2 *src, float2 *dst, int chunk, int groups, int pg,
                              hipStream_t s) {
    constexpr int TC = 1 << sh_log2_tile(LOG2H);
    const size_t lds = 2 * (size_t)TC * ((1 << LOG2H) + 1) * sizeof(float2);
    const dim3 grid((unsigned)(1 << (d.log2w - sh_log2_tile(LOG2H))), (unsigned)groups, (unsigned)chunk);
    if (!adjoint)
        hipLaunchKernelGGL((sh_cols_forward<LOG2H>), grid, dim3(kShThreads), lds, s, src, psi, dst, d.log2w,
                           d.pairs, pg, tw_h);
    else
        hipLaunchKernelGGL((sh_cols_adjoint<LOG2H>), grid, dim3(kShThreads), lds, s, src, psi, dst, d.log2w,
                           d.pairs, pg, chunk, tw_h);
    return hipGetLastError();
}

static hipError_t cols_dispatch(bool adjoint, const ShearletDims &d, const float2 *psi,
                                const float2 *tw_h, const float2 *src, float2 *dst, int chunk,
                                int groups, int pg, hipStream_t s) {
    switch (d.log2h) {
#define RADON_SH_COLS(M) \
    case M: return launch_cols<M>(adjoint, d, psi, tw_h, src, dst, chunk, groups, pg, s);
    RADON_SH_COLS(4) RADON_SH_COLS(5) RADON_SH_COLS(6) RADON_SH_COLS(7) RADON_SH_COLS(8)
    RADON_SH_COLS(9) RADON_SH_COLS(10) RADON_SH_COLS(11) RADON_SH_COLS(12)
#undef RADON_SH_COLS
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t run(bool adjoint, const ShearletDims &d, const float2 *psi, const float2 *tw_w,
                      const float2 *tw_h, const void *in, void *out, int batch, void *ws, hipStream_t s) {
    const long long plane = 1ll << (d.log2w + d.log2h);
    const long long H = 1ll << d.log2h;
    const float inv = 1.0f / (float)plane;
    const int chunk = shearlet_chunk(d, batch);
    const size_t esize = sizeof(T);
    float2 *A = (float2 *)ws;                               // X1 (forward) or U (adjoint)
    float2 *B = A + (adjoint ? (long long)chunk * d.pairs * plane : (long long)chunk * plane);
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int c = std::min(chunk, batch - b0);
        hipError_t e;
        if (!adjoint) {
            const char *x = (const char *)in + (size_t)b0 * plane * esize;
            char *co = (char *)out + (size_t)b0 * d.channels * plane * esize;
            const int groups = groups_for(d, c, d.pairs), pg = per_group(d.pairs, groups);
            if ((e = rows_dispatch<T>(false, 0, d, tw_w, x, A, c * H, 0, inv, s)) != hipSuccess) return e;
            if ((e = cols_dispatch(false, d, psi, tw_h, A, B, c, (d.pairs + pg - 1) / pg, pg, s)) != hipSuccess)
                return e;
            if ((e = rows_dispatch<T>(false, 1, d, tw_w, B, co, (long long)c * d.pairs * H, 0, inv, s)) !=
                hipSuccess)
                return e;
        } else {
            const char *co = (const char *)in + (size_t)b0 * d.channels * plane * esize;
            char *x = (char *)out + (size_t)b0 * plane * esize;
            const int pg = per_group(d.pairs, groups_for(d, chunk, 8));
            const int groups = (d.pairs + pg - 1) / pg;
            if ((e = rows_dispatch<T>(true, 0, d, tw_w, co, A, (long long)c * d.pairs * H, 0, inv, s)) !=
                hipSuccess)
                return e;
            if ((e = cols_dispatch(true, d, psi, tw_h, A, B, c, groups, pg, s)) != hipSuccess) return e;
            // the partial of group q for image ci sits at B + (q c + ci) H W: the row kernel
            // reads rows g < c H with a group stride of c H W
            if ((e = rows_dispatch<T>(true, 1, d, tw_w, B, x, c * H, groups, inv, s)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_shearlet(int dtype, bool adjoint, const ShearletDims &d, const float2 *psi,
                           const float2 *tw_w, const float2 *tw_h, const void *in, void *out,
                           int batch, void *ws, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    switch (dtype) {
    case F32: return run<float>(adjoint, d, psi, tw_w, tw_h, in, out, batch, ws, s);
    case F16: return run<__half>(adjoint, d, psi, tw_w, tw_h, in, out, batch, ws, s);
    case BF16: return run<bf16_t>(adjoint, d, psi, tw_w, tw_h, in, out, batch, ws, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
