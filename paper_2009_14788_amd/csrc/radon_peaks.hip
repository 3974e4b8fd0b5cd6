// Device calibration for the roofline fractions the benchmark reports: the FP32
// multiply-add issue rate and the LDS read bandwidth this GPU actually reaches with
// the instruction forms the projector kernels use (v_fmac_f32 with packed FP32 off;
// ds_read_b128 without bank conflicts).  Both kernels run a fixed number of
// iterations over in-bounds addresses and end.
#include <hip/hip_runtime.h>

#include "../../include/radon.h"

namespace {

constexpr int kPeakThreads = 256;
constexpr int kFmaIters = 4096;
constexpr int kFmaChains = 8;
constexpr int kLdsIters = 512;          // steps of 8 reads
constexpr int kLdsChunks = 2048;        // 32 KB of 16-byte chunks

// kFmaChains independent multiply-add chains per lane, kFmaIters steps each.
__global__ __launch_bounds__(kPeakThreads) void fma_rate(float *out, float b, float c) {
    float a[kFmaChains];
#pragma unroll
    for (int i = 0; i < kFmaChains; ++i) a[i] = (float)(threadIdx.x + i);
    for (int k = 0; k < kFmaIters; ++k) {
#pragma unroll
        for (int i = 0; i < kFmaChains; ++i) a[i] = fmaf(a[i], b, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kFmaChains; ++i) s += a[i];
    out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// Every lane reads 16-byte chunks lane-consecutively (no bank conflicts): per step 8
// chunks 4 KB apart from a base that moves every step (so no read is loop-invariant),
// kLdsIters steps, from a 32 KB buffer the block filled first; the words are folded
// with three-input adds (two VALU instructions per 16-byte read) so the reads, not the
// ALU, set the pace.
__global__ __launch_bounds__(kPeakThreads) void lds_rate(unsigned *out) {
    __shared__ uint4 buf[kLdsChunks];
    for (int i = threadIdx.x; i < kLdsChunks; i += kPeakThreads)
        buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    unsigned x = 0, y = 0, z = 0, w = 0;
    for (int k = 0; k < kLdsIters; ++k) {
        const int base = (threadIdx.x + 64 * k) & (kPeakThreads - 1);
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            const uint4 p = buf[base + kPeakThreads * u], q = buf[base + kPeakThreads * (u + 1)];
            x = x + p.x + q.x;
            y = y + p.y + q.y;
            z = z + p.z + q.z;
            w = w + p.w + q.w;
        }
    }
    out[blockIdx.x * kPeakThreads + threadIdx.x] = x + y + z + w;
}

}  // namespace

extern "C" int radon_measure_peaks(double *fma_per_s, double *lds_bytes_per_s) {
    if (!fma_per_s || !lds_bytes_per_s) return RADON_ERR_INVALID_ARG;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return RADON_ERR_NO_DEVICE;
    const int blocks = prop.multiProcessorCount * 16;
    void *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * kPeakThreads * sizeof(float)) != hipSuccess)
        return RADON_ERR_ALLOC;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = RADON_OK;
    float best_fma = 1e30f, best_lds = 1e30f;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = RADON_ERR_HIP;
    for (int rep = 0; rep < 4 && rc == RADON_OK; ++rep) {
        float ms = 0.0f;
        (void)hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(fma_rate, dim3(blocks), dim3(kPeakThreads), 0, nullptr, (float *)out,
                           0.999f, 1e-3f);
        (void)hipEventRecord(e1, nullptr);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = RADON_ERR_HIP;
            break;
        }
        if (rep > 0 && ms < best_fma) best_fma = ms;    // the first run warms the clocks
        (void)hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(lds_rate, dim3(blocks), dim3(kPeakThreads), 0, nullptr, (unsigned *)out);
        (void)hipEventRecord(e1, nullptr);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = RADON_ERR_HIP;
            break;
        }
        if (rep > 0 && ms < best_lds) best_lds = ms;
    }
    if (rc == RADON_OK) {
        const double threads = (double)blocks * kPeakThreads;
        *fma_per_s = threads * kFmaChains * kFmaIters / (best_fma * 1e-3);
        *lds_bytes_per_s = threads * kLdsIters * 8 * 16.0 / (best_lds * 1e-3);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
