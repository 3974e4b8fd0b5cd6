// Sinogram filter of filtered backprojection (TorchRadon Sec. 3.1.3): every
// projection row is zero-padded to L = 2^m >= 2D, transformed, multiplied by the
// real, even frequency response H of the chosen filter, transformed back, and the
// first D samples are kept, scaled by pi / A.  H is the transform of the
// sampled impulse response of the band-limited ramp (Kak & Slaney, ch. 3, eq. 61)
// times the filter's window; it is formed on the host in FP64.
//
// One block filters two rows at once: row 0 is the real part and row 1 the
// imaginary part of one complex sequence; because H is real and even, the filtered
// sequence's real and imaginary parts are the two filtered rows.  The transforms are
// Stockham autosort FFTs in LDS (natural order in and out, no reordering pass): radix-8
// passes with one or two radix-4 passes first when log2 L is not a multiple of 3, each
// pass a register DFT per butterfly between two barriers (4 passes for L = 2048
// instead of 11 radix-2 stages).  The inverse transform is the forward one applied to
// conj(H X), conjugated.  FP32 arithmetic; twiddles are FP64 values rounded once.
#include <cmath>

#include "radon_common.hpp"
#include "radon_fft.hpp"
#include "radon_filter.hpp"

namespace radon {

constexpr int kFilterThreads = 256;

template <typename T, int LOG2L>
__global__ __launch_bounds__(kFilterThreads) void filter_rows(const T *__restrict__ y, T *__restrict__ out,
                                                              long long rows, int D,
                                                              const float *__restrict__ H,
                                                              const float2 *__restrict__ tw, float scale) {
    extern __shared__ float2 buf[];
    constexpr int L = 1 << LOG2L;
    const long long r0 = 2 * (long long)blockIdx.x;
    const bool has1 = r0 + 1 < rows;
    const T *y0 = y + r0 * D;
    const T *y1 = y + (has1 ? r0 + 1 : r0) * D;
    for (int k = threadIdx.x; k < L; k += kFilterThreads) {
        float2 v = make_float2(0.0f, 0.0f);
        if (k < D) {
            v.x = Store<T>::load(y0 + k);
            v.y = has1 ? Store<T>::load(y1 + k) : 0.0f;
        }
        buf[k] = v;
    }
    __syncthreads();
    fft_multi<kFilterThreads, 1, L, LOG2L>(buf, tw);
    // conj(X) H: the inverse transform is conj(FFT(conj(H X))) / L
    for (int k = threadIdx.x; k < L; k += kFilterThreads) {
        const float h = H[k];
        const float2 x = buf[k];
        buf[k] = make_float2(x.x * h, -x.y * h);
    }
    __syncthreads();
    fft_multi<kFilterThreads, 1, L, LOG2L>(buf, tw);
    const float f = scale / (float)L;
    T *o0 = out + r0 * D;
    T *o1 = out + (r0 + 1) * D;
    for (int n = threadIdx.x; n < D; n += kFilterThreads) {
        const float2 v = buf[n];
        Store<T>::store(o0 + n, v.x * f);
        if (has1) Store<T>::store(o1 + n, -v.y * f);
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
    tw.resize(L);
    for (int k = 0; k < L; ++k)
        tw[k] = make_float2((float)std::cos(2.0 * pi * k / L), (float)-std::sin(2.0 * pi * k / L));
}

template <typename T>
static hipError_t launch_rows(const void *y, void *out, long long rows, int D, int log2L,
                              const float *H, const float2 *tw, float scale, hipStream_t s) {
    const size_t lds = sizeof(float2) << log2L;
    const dim3 grid((unsigned)((rows + 1) / 2)), block(kFilterThreads);
    const T *yi = (const T *)y;
    T *o = (T *)out;
    switch (log2L) {
#define RADON_FILTER_CASE(M) \
    case M: hipLaunchKernelGGL((filter_rows<T, M>), grid, block, lds, s, yi, o, rows, D, H, tw, scale); break;
    RADON_FILTER_CASE(6) RADON_FILTER_CASE(7) RADON_FILTER_CASE(8) RADON_FILTER_CASE(9)
    RADON_FILTER_CASE(10) RADON_FILTER_CASE(11) RADON_FILTER_CASE(12) RADON_FILTER_CASE(13)
#undef RADON_FILTER_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_filter(int dtype, const void *y, void *out, long long rows, int D, int log2L,
                         const float *H, const float2 *tw, float scale, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if ((rows + 1) / 2 > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (dtype) {
    case F32: return launch_rows<float>(y, out, rows, D, log2L, H, tw, scale, s);
    case F16: return launch_rows<__half>(y, out, rows, D, log2L, H, tw, scale, s);
    case BF16: return launch_rows<bf16_t>(y, out, rows, D, log2L, H, tw, scale, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
