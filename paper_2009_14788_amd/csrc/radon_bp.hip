// Backprojection kernels: x[b][r][c] = scale * sum_{a,d} R[(a,d),(r,c)] * y[b][a][d].
//
// The exact transpose of the forward projection (TorchRadon uses it as the adjoint
// inside its CG solver, Sec. 4.3), computed as a gather: each thread owns pixels
// and collects, per angle, every sample of every ray whose bilinear footprint
// covers the pixel.  No atomics; results are deterministic.
#include "radon_common.hpp"
#include "radon_launch.hpp"

namespace radon {

// Bins [dlo, dhi] whose rays can pass through the 2x2-pixel footprint of the pixel
// with centred coordinates (qx, qy) at angle cs = (cos, sin).  A sample inside the
// footprint differs from the pixel centre by less than 1 in x and in y, so its
// detector coordinate is within |cos|+|sin| (parallel), or between the projections
// of the footprint corners (fan), of the pixel's.  The 1e-3 margin covers FP32
// rounding of the sample positions.
__device__ __forceinline__ void bin_window(const Geom &g, float qx, float qy, float2 cs,
                                           int &dlo, int &dhi) {
    float lo, hi;
    if (!g.fan) {
        const float t = fmaf(qx, cs.x, qy * cs.y);
        const float h = fabsf(cs.x) + fabsf(cs.y);
        lo = (t - h) * g.inv_spacing + g.half_d;
        hi = (t + h) * g.inv_spacing + g.half_d;
    } else {
        lo = 3.0e7f;
        hi = -3.0e7f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float px = qx + ((j & 1) ? 1.0f : -1.0f);
            const float py = qy + ((j & 2) ? 1.0f : -1.0f);
            const float pu = fmaf(px, cs.x, py * cs.y);
            const float pv = fmaf(-px, cs.y, py * cs.x);
            const float s = g.sde * pu / (g.sd + pv) * g.inv_spacing + g.half_d;
            lo = fminf(lo, s);
            hi = fmaxf(hi, s);
        }
    }
    dlo = max(0, (int)ceilf(lo - 1e-3f));
    dhi = min(g.det_count - 1, (int)floorf(hi + 1e-3f));
}

// Sum over the samples k of ray rp of the bilinear weight they give pixel (rf, cf).
__device__ __forceinline__ float footprint_weight(const Geom &g, const float4 &rp, float cf,
                                                  float rf) {
    const float is2 = g.inv_step * g.inv_step;
    const float kc = fmaf(cf - rp.x, rp.z, (rf - rp.y) * rp.w) * is2;
    const float hk = (fabsf(rp.z) + fabsf(rp.w)) * is2;
    const int klo = (int)ceilf(kc - hk - 1e-3f), khi = (int)floorf(kc + hk + 1e-3f);
    float w = 0.0f;
    for (int k = klo; k <= khi; ++k) {
        const float kf = (float)k;
        const float px = fmaf(kf, rp.z, rp.x), py = fmaf(kf, rp.w, rp.y);
        w += __fmul_rn(tent(px, cf), tent(py, rf));
    }
    return w;
}

// Direct variant: one thread per (pixel, group of BC images), 16x16 pixel tiles;
// sinogram values are read from global memory through the caches.
template <typename T, int BC>
__global__ __launch_bounds__(256) void bp_direct(Geom g, const T *__restrict__ y,
                                                 T *__restrict__ x, int batch, float scale) {
    const int c = blockIdx.x * 16 + (threadIdx.x & 15);
    const int r = blockIdx.y * 16 + (threadIdx.x >> 4);
    const int b0 = blockIdx.z * BC;
    const int n = g.n;
    if (c >= n || r >= n) return;
    const float cf = (float)c, rf = (float)r;
    const float qx = cf - g.cn, qy = rf - g.cn;
    const size_t sino = (size_t)g.n_angles * g.det_count;

    const T *src[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) src[i] = y + (size_t)min(b0 + i, batch - 1) * sino;

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int a = 0; a < g.n_angles; ++a) {
        const float2 cs = g.trig[a];
        int dlo, dhi;
        bin_window(g, qx, qy, cs, dlo, dhi);
        const size_t row = (size_t)a * g.det_count;
        for (int d = dlo; d <= dhi; ++d) {
            const float w = footprint_weight(g, ray_params(g, a, d), cf, rf);
#pragma unroll
            for (int i = 0; i < BC; ++i) acc[i] = fmaf(w, Store<T>::load(src[i] + row + d), acc[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < BC; ++i) {
        if (b0 + i < batch)
            Store<T>::store(x + (size_t)(b0 + i) * n * n + (size_t)r * n + c, acc[i] * scale);
    }
}

template <typename T, int BC>
static hipError_t launch_bp_direct(const Geom &g, const void *y, void *x, int batch, float scale,
                                   hipStream_t s) {
    dim3 block(256);
    dim3 grid((g.n + 15) / 16, (g.n + 15) / 16, (batch + BC - 1) / BC);
    hipLaunchKernelGGL((bp_direct<T, BC>), grid, block, 0, s, g, (const T *)y, (T *)x, batch,
                       scale);
    return hipGetLastError();
}

hipError_t launch_backproject(const Geom &g, int dtype, const LaunchShape &shape, const void *y,
                              void *x, int batch, float scale, hipStream_t s) {
    (void)shape;
    switch (dtype) {
    case F32: return launch_bp_direct<float, 4>(g, y, x, batch, scale, s);
    case F16: return launch_bp_direct<__half, 4>(g, y, x, batch, scale, s);
    case BF16: return launch_bp_direct<bf16_t, 4>(g, y, x, batch, scale, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
