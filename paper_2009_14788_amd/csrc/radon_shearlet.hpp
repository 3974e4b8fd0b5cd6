// Host interface of the alpha-shearlet transform kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace radon {

constexpr int kShMinLog2 = 4;    // image sides 16 .. 4096 (powers of two)
constexpr int kShMaxLog2 = 12;

// Layout of one shearlet plan on the device.
struct ShearletDims {
    int log2w = 0, log2h = 0;
    int channels = 0;      // M
    int pairs = 0;         // P = ceil(M / 2): channels 2p and 2p + 1 travel as one complex field
};

// Filters psi_m[k1][k2] (k1 row frequency, k2 column frequency, FFT order), FP64 on
// the host, for an image of width 2^log2w and height 2^log2h and one alpha per scale;
// out[m * H * W + k1 * W + k2].  Returns the channel count M.
int shearlet_filters(int width, int height, const std::vector<double> &alphas,
                     std::vector<double> &out);
// Channel count and each channel's scale (0 = low-pass, j + 1 = scale j).
int shearlet_channels(const std::vector<double> &alphas, std::vector<int> *scales);

// Bytes of stream workspace one call needs for a chunk of `chunk` images.
size_t shearlet_workspace_bytes(const ShearletDims &d, int chunk, bool adjoint);
// Images per chunk for a batch (bounded so the intermediate fields stay <= ~512 MB).
int shearlet_chunk(const ShearletDims &d, int batch);

// Forward: coeffs[b][m][H][W] = Re IFFT2(FFT2(x[b]) psi_m); adjoint: x[b] =
// Re IFFT2(sum_m FFT2(coeffs[b][m]) psi_m).  psi: device [P][W][H] float2 (channel 2p
// in .x, 2p + 1 in .y, column-major per pair); tw_w, tw_h: device twiddle tables of
// lengths W and H.  ws: device workspace of shearlet_workspace_bytes(d, chunk, ...).
hipError_t launch_shearlet(int dtype, bool adjoint, const ShearletDims &d, const float2 *psi,
                           const float2 *tw_w, const float2 *tw_h, const void *in, void *out,
                           int batch, void *ws, hipStream_t s);

}  // namespace radon
