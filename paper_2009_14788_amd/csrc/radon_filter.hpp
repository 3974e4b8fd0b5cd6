// Host interface of the FBP sinogram filter kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace radon {

enum FilterKind { FILTER_RAMLAK = 0, FILTER_SHEPP_LOGAN = 1, FILTER_COSINE = 2, FILTER_HAMMING = 3,
                  FILTER_HANN = 4 };
constexpr int kFilterMaxLog2 = 13;   // L <= 8192: the row pair's transform fits in 64 KB of LDS

// log2 of the padded row length L: the smallest power of two >= max(64, 2 D).
int filter_log2_length(int det_count);
// Frequency response H[0..L) of a filter (FP64 on the host, rounded to FP32).
void filter_response(int filter, int log2L, std::vector<float> &H);
// Forward twiddles exp(-2 pi i k / L), k < L.
void filter_twiddles(int log2L, std::vector<float2> &tw);
// out[r][0..D) = scale * (row r of y filtered by H), for `rows` rows of D values of
// `dtype` (in place allowed: out == y).
hipError_t launch_filter(int dtype, const void *y, void *out, long long rows, int D, int log2L,
                         const float *H, const float2 *tw, float scale, hipStream_t s);

}  // namespace radon
