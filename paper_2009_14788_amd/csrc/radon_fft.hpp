// Radix-4/8 Stockham FFT building blocks in LDS (FP32 complex as float2), used by the
// FBP sinogram filter and the shearlet transform.  Forward transforms
// X_k = sum_n x_n exp(-2 pi i n k / L), natural order in and out; an inverse transform
// is the forward one applied to the conjugate, conjugated (and divided by L).
// Twiddles come from a table tw[k] = exp(-2 pi i k / L), k < L, formed in FP64 on the
// host and rounded once.
#pragma once

#include <hip/hip_runtime.h>

namespace radon {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// In-register DFTs, natural order in and out.
__device__ __forceinline__ void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3) {
    const float2 a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = csub(x1, x3);
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = make_float2(b.x + d.y, b.y - d.x);             // b - i d
    x3 = make_float2(b.x - d.y, b.y + d.x);             // b + i d
}

template <int R> __device__ __forceinline__ void dft(float2 *v);

template <> __device__ __forceinline__ void dft<4>(float2 *v) { dft4(v[0], v[1], v[2], v[3]); }

template <> __device__ __forceinline__ void dft<8>(float2 *v) {
    // even and odd halves, then X_k = E_k + W^k O_k, X_{k+4} = E_k - W^k O_k, W = exp(-i pi/4)
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    constexpr float c = 0.70710678118654752f;
    const float2 t1 = make_float2(c * (o1.x + o1.y), c * (o1.y - o1.x));    // W   o1
    const float2 t2 = make_float2(o2.y, -o2.x);                            // W^2 o2 = -i o2
    const float2 t3 = make_float2(c * (o3.y - o3.x), -c * (o3.x + o3.y));   // W^3 o3
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1);
    v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2);
    v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3);
    v[7] = csub(e3, t3);
}

// One Stockham pass of radix R = 2^LOG2R over NSEQ sequences of length L = 2^LOG2L held
// in LDS at buf + s * STRIDE, done by THREADS threads together, Ns = 2^LOG2NS: every
// thread first reads all its butterflies' inputs, the block synchronises, then each
// butterfly j of sequence s (k = j mod Ns) applies the twiddles
// exp(-2 pi i r k / (Ns R)) = tw[r k L / (Ns R)], its R-point DFT, and writes output r
// to (j - k) R + k + r Ns.  Ends with a block barrier.
template <int THREADS, int NSEQ, int STRIDE, int LOG2R, int LOG2L, int LOG2NS>
__device__ __forceinline__ void stockham_pass_multi(float2 *buf, const float2 *__restrict__ tw) {
    constexpr int R = 1 << LOG2R;
    constexpr int LOG2NB = LOG2L - LOG2R;
    constexpr int nb = 1 << LOG2NB;                       // butterflies per sequence
    constexpr int Ns = 1 << LOG2NS;
    constexpr int sh = LOG2L - LOG2NS - LOG2R;
    constexpr int total = nb * NSEQ;
    constexpr int JMAX = (total + THREADS - 1) / THREADS;
    float2 v[JMAX][R];
#pragma unroll
    for (int jj = 0; jj < JMAX; ++jj) {
        const int idx = threadIdx.x + THREADS * jj;
        if (total % THREADS == 0 || idx < total) {
            const float2 *b = buf + (idx >> LOG2NB) * STRIDE + (idx & (nb - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) v[jj][r] = b[r * nb];
        }
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < JMAX; ++jj) {
        const int idx = threadIdx.x + THREADS * jj;
        if (total % THREADS == 0 || idx < total) {
            const int j = idx & (nb - 1);
            const int k = j & (Ns - 1);
            if (Ns > 1 && k != 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[jj][r] = cmul(v[jj][r], tw[(r * k) << sh]);
            }
            dft<R>(v[jj]);
            float2 *b = buf + (idx >> LOG2NB) * STRIDE + ((j - k) << LOG2R) + k;
#pragma unroll
            for (int r = 0; r < R; ++r) b[r * Ns] = v[jj][r];
        }
    }
    __syncthreads();
}

// Forward transforms of NSEQ sequences of length 2^LOG2L (LOG2L >= 2) in place: radix-4
// passes while the remaining exponent is not a multiple of 3, then radix-8 passes.
// The caller synchronises the block before the first pass reads buf.
template <int THREADS, int NSEQ, int STRIDE, int LOG2L, int LOG2NS = 0>
__device__ __forceinline__ void fft_multi(float2 *buf, const float2 *__restrict__ tw) {
    if constexpr (LOG2NS < LOG2L) {
        constexpr int LOG2R = (LOG2L - LOG2NS) % 3 != 0 ? 2 : 3;
        stockham_pass_multi<THREADS, NSEQ, STRIDE, LOG2R, LOG2L, LOG2NS>(buf, tw);
        fft_multi<THREADS, NSEQ, STRIDE, LOG2L, LOG2NS + LOG2R>(buf, tw);
    }
}

}  // namespace radon
