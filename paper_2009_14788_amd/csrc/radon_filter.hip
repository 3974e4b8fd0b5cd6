// Sinogram filter of filtered backprojection (TorchRadon Sec. 3.1.3): every
// projection row is zero-padded to L = 2^m >= 2D, transformed, multiplied by the
// real, even frequency response H of the chosen filter, transformed back, and the
// first D samples are kept, scaled by pi / (A * spacing).  H is the transform of the
// sampled impulse response of the band-limited ramp (Kak & Slaney, ch. 3, eq. 61)
// times the filter's window; it is formed on the host in FP64.
//
// One block filters two rows at once: row 0 is the real part and row 1 the
// imaginary part of one complex sequence; because H is real and even, the filtered
// sequence's real and imaginary parts are the two filtered rows.  The transforms are
// radix-2 in LDS: decimation in time from bit-reversed input for the forward
// transform, decimation in frequency with conjugate twiddles for the inverse, so no
// reordering pass is needed.  FP32 arithmetic; twiddles are FP64 values rounded once.
#include <cmath>

#include "radon_common.hpp"
#include "radon_filter.hpp"

namespace radon {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

template <typename T>
__global__ __launch_bounds__(256) void filter_rows(const T *__restrict__ y, T *__restrict__ out,
                                                   long long rows, int D, int log2L,
                                                   const float *__restrict__ H,
                                                   const float2 *__restrict__ tw, float scale) {
    extern __shared__ float2 buf[];
    const int L = 1 << log2L;
    const long long r0 = 2 * (long long)blockIdx.x;
    const bool has1 = r0 + 1 < rows;
    const T *y0 = y + r0 * D;
    const T *y1 = y + (has1 ? r0 + 1 : r0) * D;
    // bit-reversed load: buf[k] = x[brev(k)]
    for (int k = threadIdx.x; k < L; k += 256) {
        const int j = (int)(__brev((unsigned)k) >> (32 - log2L));
        float2 v = make_float2(0.0f, 0.0f);
        if (j < D) {
            v.x = Store<T>::load(y0 + j);
            v.y = has1 ? Store<T>::load(y1 + j) : 0.0f;
        }
        buf[k] = v;
    }
    __syncthreads();
    // forward transform, decimation in time: spans 1, 2, 4, ...
    for (int s = 1; s <= log2L; ++s) {
        const int half = 1 << (s - 1);
        for (int b = threadIdx.x; b < (L >> 1); b += 256) {
            const int pos = b & (half - 1);
            const int i0 = ((b >> (s - 1)) << s) + pos, i1 = i0 + half;
            const float2 w = tw[pos << (log2L - s)];           // exp(-2 pi i pos / (2 half))
            const float2 a = buf[i0], t = cmul(buf[i1], w);
            buf[i0] = make_float2(a.x + t.x, a.y + t.y);
            buf[i1] = make_float2(a.x - t.x, a.y - t.y);
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < L; k += 256) {
        const float h = H[k];
        buf[k] = make_float2(buf[k].x * h, buf[k].y * h);
    }
    __syncthreads();
    // inverse transform, decimation in frequency with conjugate twiddles: spans
    // L/2, ..., 1; the result ends in bit-reversed order
    for (int s = log2L; s >= 1; --s) {
        const int half = 1 << (s - 1);
        for (int b = threadIdx.x; b < (L >> 1); b += 256) {
            const int pos = b & (half - 1);
            const int i0 = ((b >> (s - 1)) << s) + pos, i1 = i0 + half;
            const float2 w = tw[pos << (log2L - s)];
            const float2 wc = make_float2(w.x, -w.y);          // exp(+2 pi i pos / (2 half))
            const float2 a = buf[i0], c = buf[i1];
            buf[i0] = make_float2(a.x + c.x, a.y + c.y);
            buf[i1] = cmul(make_float2(a.x - c.x, a.y - c.y), wc);
        }
        __syncthreads();
    }
    const float f = scale / (float)L;
    T *o0 = out + r0 * D;
    T *o1 = out + (r0 + 1) * D;
    for (int n = threadIdx.x; n < D; n += 256) {
        const float2 v = buf[__brev((unsigned)n) >> (32 - log2L)];
        Store<T>::store(o0 + n, v.x * f);
        if (has1) Store<T>::store(o1 + n, v.y * f);
    }
}

int filter_log2_length(int det_count) {
    int m = 6;
    while ((1 << m) < 2 * det_count) ++m;
    return m;
}

// H[k] for k < L: the ramp's response is the cosine series of the even impulse
// response h(0) = 1/4, h(+-m) = -1/(pi^2 m^2) for odd m (|m| < L/2), 0 otherwise;
// the window is a function of the normalised frequency f in [-1/2, 1/2).
void filter_response(int filter, int log2L, std::vector<float> &H) {
    const int L = 1 << log2L;
    const double pi = 3.14159265358979323846;
    H.assign(L, 0.0f);
    for (int k = 0; k < L; ++k) {
        double r = 0.25;
        for (int m = 1; m < L / 2; m += 2)
            r -= 2.0 / (pi * pi * (double)m * m) * std::cos(2.0 * pi * (double)k * m / L);
        const double f = (k < L / 2 ? k : k - L) / (double)L;
        double w = 1.0;
        switch (filter) {
        case FILTER_SHEPP_LOGAN: w = f == 0.0 ? 1.0 : std::sin(pi * f) / (pi * f); break;
        case FILTER_COSINE: w = std::cos(pi * f); break;
        case FILTER_HAMMING: w = 0.54 + 0.46 * std::cos(2.0 * pi * f); break;
        case FILTER_HANN: w = 0.5 + 0.5 * std::cos(2.0 * pi * f); break;
        default: break;
        }
        H[k] = (float)(r * w);
    }
}

void filter_twiddles(int log2L, std::vector<float2> &tw) {
    const int L = 1 << log2L;
    const double pi = 3.14159265358979323846;
    tw.resize(L / 2);
    for (int k = 0; k < L / 2; ++k)
        tw[k] = make_float2((float)std::cos(2.0 * pi * k / L), (float)-std::sin(2.0 * pi * k / L));
}

hipError_t launch_filter(int dtype, const void *y, void *out, long long rows, int D, int log2L,
                         const float *H, const float2 *tw, float scale, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const size_t lds = sizeof(float2) << log2L;
    const long long blocks = (rows + 1) / 2;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (dtype) {
    case F32:
        hipLaunchKernelGGL(filter_rows<float>, dim3((unsigned)blocks), dim3(256), lds, s,
                           (const float *)y, (float *)out, rows, D, log2L, H, tw, scale);
        break;
    case F16:
        hipLaunchKernelGGL(filter_rows<__half>, dim3((unsigned)blocks), dim3(256), lds, s,
                           (const __half *)y, (__half *)out, rows, D, log2L, H, tw, scale);
        break;
    case BF16:
        hipLaunchKernelGGL(filter_rows<bf16_t>, dim3((unsigned)blocks), dim3(256), lds, s,
                           (const bf16_t *)y, (bf16_t *)out, rows, D, log2L, H, tw, scale);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace radon
