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
// detector coordinate is within |cos|+|sin| of the pixel's (parallel), or between
// the projections of the footprint corners (fan).  The margin covers rounding.
__device__ __forceinline__ void bin_window(const Geom &g, double qx, double qy, double2 cs,
                                           int &dlo, int &dhi) {
    double lo, hi;
    if (!g.fan) {
        const double t = fma(qx, cs.x, qy * cs.y);
        const double h = fabs(cs.x) + fabs(cs.y);
        lo = (t - h) * g.inv_spacing + g.half_d;
        hi = (t + h) * g.inv_spacing + g.half_d;
    } else {
        lo = 1.0e9;
        hi = -1.0e9;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double px = qx + ((j & 1) ? 1.0 : -1.0);
            const double py = qy + ((j & 2) ? 1.0 : -1.0);
            const double pu = fma(px, cs.x, py * cs.y);
            const double pv = fma(-px, cs.y, py * cs.x);
            const double s = g.sde * pu / (g.sd + pv) * g.inv_spacing + g.half_d;
            lo = fmin(lo, s);
            hi = fmax(hi, s);
        }
    }
    dlo = max(0, (int)ceil(lo - 1e-6));
    dhi = min(g.det_count - 1, (int)floor(hi + 1e-6));
}

// Sum over the samples k of ray rp of the bilinear weight they give pixel (r, c),
// with the sample positions and FP32 weights formed exactly as in the forward kernel.
__device__ __forceinline__ float footprint_weight(const Geom &g, const double4 &rp, int c, int r) {
    const double is2 = g.inv_step * g.inv_step;
    const double kc = fma((double)c - rp.x, rp.z, ((double)r - rp.y) * rp.w) * is2;
    const double hk = (fabs(rp.z) + fabs(rp.w)) * is2;
    const int klo = (int)ceil(kc - hk - 1e-6), khi = (int)floor(kc + hk + 1e-6);
    float w = 0.0f;
    for (int k = klo; k <= khi; ++k) {
        const double kd = (double)k;
        const Cell cx = cell_of(fma(kd, rp.z, rp.x)), cy = cell_of(fma(kd, rp.w, rp.y));
        w += __fmul_rn(axis_weight(cx, c), axis_weight(cy, r));
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
    const double qx = (double)c - g.cn, qy = (double)r - g.cn;
    const size_t sino = (size_t)g.n_angles * g.det_count;

    const T *src[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) src[i] = y + (size_t)min(b0 + i, batch - 1) * sino;

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int a = 0; a < g.n_angles; ++a) {
        const double2 cs = g.trig[a];
        int dlo, dhi;
        bin_window(g, qx, qy, cs, dlo, dhi);
        const size_t row = (size_t)a * g.det_count;
        for (int d = dlo; d <= dhi; ++d) {
            const float w = footprint_weight(g, ray_params(g, a, d), c, r);
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

// ------------------------------------------------------------------ tiled variant
// Parallel beam.  One block = a 16x16 pixel tile (lane <-> pixel) x BC images.
// Angles are processed in blocks of kBpAngles: for each, the block stages into LDS
// the window of W bins its tile can touch, as 16-byte chunks of Chunk<T>::kImages
// images ("planes").  Each pixel then finds, per angle, the lattice samples
// (bin d, step k) whose bilinear footprint covers it: the pixel's continuous
// lattice coordinates (u*, v*) are formed in FP64, the NB x NK candidates
// d = floor(u* - hu) + 1 + i, k = floor(v* - hv) + 1 + j cover every sample within
// the footprint, and their offsets from the pixel are small FP32 numbers, so the
// tent weights are accurate to FP32 rounding.  The NB bin weights are then applied
// to BC images with 16-byte LDS reads.  No atomics.
template <typename T, int BC, int NB, int NK>
__global__ __launch_bounds__(256) void bp_tiled_par(Geom g, const T *__restrict__ y,
                                                    T *__restrict__ x, int batch, float scale_dt,
                                                    int W) {
    extern __shared__ uint4 lds[];
    __shared__ int wlo_s[kBpAngles];
    constexpr int CH = Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    static_assert(BC % CH == 0, "BC must be a multiple of the images per chunk");
    const int n = g.n, A = g.n_angles, D = g.det_count;
    const int tiles_x = (n + kBpTile - 1) / kBpTile;
    const int tx0 = (blockIdx.x % tiles_x) * kBpTile, ty0 = (blockIdx.x / tiles_x) * kBpTile;
    const int c = tx0 + (threadIdx.x % kBpTile), r = ty0 + (threadIdx.x / kBpTile);
    const int b0 = blockIdx.y * BC;
    const double qx = (double)c - g.cn, qy = (double)r - g.cn;
    const double tcx = tx0 + 0.5 * (kBpTile - 1) - g.cn, tcy = ty0 + 0.5 * (kBpTile - 1) - g.cn;
    const size_t sino = (size_t)A * D;
    const int per_plane = kBpAngles * W;
    const T *img_base[BC];
#pragma unroll
    for (int e = 0; e < BC; ++e) img_base[e] = y + (size_t)min(b0 + e, batch - 1) * sino;
    const float dt = (float)g.step, sp = (float)g.spacing;

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int a0 = 0; a0 < A; a0 += kBpAngles) {
        const int na = min(kBpAngles, A - a0);
        __syncthreads();                                // previous block consumed
        if (threadIdx.x < na) {
            const double2 cs = g.trig[a0 + threadIdx.x];
            const double h = fabs(cs.x) + fabs(cs.y);
            const double uc = fma(fma(tcx, cs.x, tcy * cs.y), g.inv_spacing, g.half_d);
            wlo_s[threadIdx.x] = (int)floor(uc - (0.5 * (kBpTile - 1) + 1.0) * h * g.inv_spacing) - 1;
        }
        __syncthreads();
        for (int p = threadIdx.x; p < na * W; p += 256) {
            const int al = p / W, j = p - al * W;
            const int d = wlo_s[al] + j;
            const bool inside = (unsigned)d < (unsigned)D;
            const unsigned off = (unsigned)((a0 + al) * D + (inside ? d : 0));
#pragma unroll
            for (int q = 0; q < PLANES; ++q) {
                T v[CH];
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    const T val = img_base[q * CH + e][off];   // always a valid address
                    v[e] = inside ? val : Chunk<T>::zero();
                }
                lds[q * per_plane + al * W + j] = Chunk<T>::pack(v);
            }
        }
        __syncthreads();

        // the angle block's contributions are summed separately, then added to the
        // pixel total (two-level summation keeps FP32 rounding small)
        float part[BC];
#pragma unroll
        for (int i = 0; i < BC; ++i) part[i] = 0.0f;
        for (int al = 0; al < na; ++al) {
            const double2 cs = g.trig[a0 + al];
            const double h = fabs(cs.x) + fabs(cs.y);
            // continuous bin (u) and step (v) coordinates of the pixel centre
            const double u = fma(fma(qx, cs.x, qy * cs.y), g.inv_spacing, g.half_d);
            const double v = fma(qy, cs.x, -qx * cs.y) * g.inv_step;
            const double db = floor(u - h * g.inv_spacing), kb = floor(v - h * g.inv_step);
            // offset of candidate (d = db+1+i, k = kb+1+j) from the pixel, along u and v
            const float e0 = (float)(db + 1.0 - u) * sp, t0 = (float)(kb + 1.0 - v) * dt;
            const float cf = (float)cs.x, sf = (float)cs.y;
            const float ux = sp * cf, uy = sp * sf;      // one bin along u
            const float vx = -dt * sf, vy = dt * cf;     // one step along v
            float dx_i = fmaf(e0, cf, -t0 * sf), dy_i = fmaf(e0, sf, t0 * cf);
            float wgt[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                float dx = dx_i, dy = dy_i, w = 0.0f;
#pragma unroll
                for (int jj = 0; jj < NK; ++jj) {
                    const float tx = __builtin_amdgcn_fmed3f(1.0f - fabsf(dx), 0.0f, 1.0f);
                    const float ty = __builtin_amdgcn_fmed3f(1.0f - fabsf(dy), 0.0f, 1.0f);
                    w = fmaf(tx, ty, w);
                    dx += vx;
                    dy += vy;
                }
                wgt[i] = w;
                dx_i += ux;
                dy_i += uy;
            }
            int lb = (int)db + 1 - wlo_s[al];
            lb = min(max(lb, 0), W - NB);               // memory safety; real pixels are inside
            const uint4 *row = lds + al * W + lb;
#pragma unroll
            for (int qq = 0; qq < PLANES; ++qq) {
#pragma unroll
                for (int i = 0; i < NB; ++i) Chunk<T>::fma(wgt[i], row[qq * per_plane + i], part + qq * CH);
            }
        }
#pragma unroll
        for (int i = 0; i < BC; ++i) acc[i] += part[i];
    }
    if (c >= n || r >= n) return;
#pragma unroll
    for (int i = 0; i < BC; ++i)
        if (b0 + i < batch)
            Store<T>::store(x + (size_t)(b0 + i) * n * n + (size_t)r * n + c, acc[i] * scale_dt);
}

// Fan beam.  Same tiling as the parallel kernel; every bin has its own ray, so the
// block also stages the rays (FP64 foot point and step) of its bin window.  Per
// (pixel, angle) the candidate bins are those within the projected half-width of
// the pixel's footprint around the projection of its centre (first-order bound
// plus a margin far larger than the footprint's curvature); per bin, the NK
// candidate samples around the pixel's position along that ray are evaluated with
// FP64 anchors and FP32 offsets, exactly as in the parallel kernel.
template <typename T, int BC, int NB, int NK>
__global__ __launch_bounds__(256) void bp_tiled_fan(Geom g, const T *__restrict__ y,
                                                    T *__restrict__ x, int batch, float scale_dt,
                                                    int W) {
    extern __shared__ uint4 lds[];
    __shared__ int wlo_s[kBpAnglesFan];
    constexpr int CH = Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    static_assert(BC % CH == 0, "BC must be a multiple of the images per chunk");
    const int n = g.n, A = g.n_angles, D = g.det_count;
    const int tiles_x = (n + kBpTile - 1) / kBpTile;
    const int tx0 = (blockIdx.x % tiles_x) * kBpTile, ty0 = (blockIdx.x / tiles_x) * kBpTile;
    const int c = tx0 + (threadIdx.x % kBpTile), r = ty0 + (threadIdx.x / kBpTile);
    const int b0 = blockIdx.y * BC;
    const double qx = (double)c - g.cn, qy = (double)r - g.cn;
    const size_t sino = (size_t)A * D;
    const int per_plane = kBpAnglesFan * W;
    double4 *rays_s = reinterpret_cast<double4 *>(lds + PLANES * per_plane);
    const T *img_base[BC];
#pragma unroll
    for (int e = 0; e < BC; ++e) img_base[e] = y + (size_t)min(b0 + e, batch - 1) * sino;
    const double is2 = g.inv_step * g.inv_step;

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int a0 = 0; a0 < A; a0 += kBpAnglesFan) {
        const int na = min(kBpAnglesFan, A - a0);
        __syncthreads();
        if (threadIdx.x < na) {
            // bin window of the tile: projections of the corners of its footprint
            const double2 cs = g.trig[a0 + threadIdx.x];
            double lo = 1e30;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double px = tx0 - 1.0 + ((k & 1) ? kBpTile + 1.0 : 0.0) - g.cn;
                const double py = ty0 - 1.0 + ((k & 2) ? kBpTile + 1.0 : 0.0) - g.cn;
                const double pu = fma(px, cs.x, py * cs.y), pv = fma(-px, cs.y, py * cs.x);
                lo = fmin(lo, g.sde * pu / (g.sd + pv) * g.inv_spacing + g.half_d);
            }
            wlo_s[threadIdx.x] = (int)floor(lo) - 1;
        }
        __syncthreads();
        for (int p = threadIdx.x; p < na * W; p += 256) {
            const int al = p / W, j = p - al * W;
            const int d = wlo_s[al] + j;
            const bool inside = (unsigned)d < (unsigned)D;
            const unsigned off = (unsigned)((a0 + al) * D + (inside ? d : 0));
#pragma unroll
            for (int q = 0; q < PLANES; ++q) {
                T v[CH];
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    const T val = img_base[q * CH + e][off];
                    v[e] = inside ? val : Chunk<T>::zero();
                }
                lds[q * per_plane + al * W + j] = Chunk<T>::pack(v);
            }
            // a bin outside the detector gets a ray far from every pixel (weight 0)
            rays_s[al * W + j] = inside ? g.rays[off] : make_double4(-1e9, -1e9, 0.0, 0.0);
        }
        __syncthreads();

        float part[BC];
#pragma unroll
        for (int i = 0; i < BC; ++i) part[i] = 0.0f;
        for (int al = 0; al < na; ++al) {
            const double2 cs = g.trig[a0 + al];
            // detector coordinate of the pixel centre and its gradient (bins per pixel)
            const double pu = fma(qx, cs.x, qy * cs.y), pv = fma(-qx, cs.y, qy * cs.x);
            const double den = 1.0 / (g.sd + pv);
            const double sb = g.sde * pu * den * g.inv_spacing + g.half_d;
            const double gsx = g.sde * (cs.x * (g.sd + pv) + pu * cs.y) * den * den * g.inv_spacing;
            const double gsy = g.sde * (cs.y * (g.sd + pv) - pu * cs.x) * den * den * g.inv_spacing;
            const double hb = fabs(gsx) + fabs(gsy);
            const int dfirst = (int)ceil(sb - hb * 1.01 - 0.05);
            int lb = dfirst - wlo_s[al];
            lb = min(max(lb, 0), W - NB);               // memory safety; real pixels are inside
            float wgt[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const double4 rp = rays_s[al * W + lb + i];
                const double ex = rp.x - (double)c, ey = rp.y - (double)r;   // F - Q
                const double kc = -fma(ex, rp.z, ey * rp.w) * is2;           // pixel along the ray
                const double hk = (fabs(rp.z) + fabs(rp.w)) * is2;
                const double k0 = floor(kc - hk);
                float dx = (float)fma(k0 + 1.0, rp.z, ex), dy = (float)fma(k0 + 1.0, rp.w, ey);
                const float sx = (float)rp.z, sy = (float)rp.w;
                float w = 0.0f;
#pragma unroll
                for (int jj = 0; jj < NK; ++jj) {
                    const float tx = __builtin_amdgcn_fmed3f(1.0f - fabsf(dx), 0.0f, 1.0f);
                    const float ty = __builtin_amdgcn_fmed3f(1.0f - fabsf(dy), 0.0f, 1.0f);
                    w = fmaf(tx, ty, w);
                    dx += sx;
                    dy += sy;
                }
                wgt[i] = w;
            }
            const uint4 *row = lds + al * W + lb;
#pragma unroll
            for (int qq = 0; qq < PLANES; ++qq) {
#pragma unroll
                for (int i = 0; i < NB; ++i) Chunk<T>::fma(wgt[i], row[qq * per_plane + i], part + qq * CH);
            }
        }
#pragma unroll
        for (int i = 0; i < BC; ++i) acc[i] += part[i];
    }
    if (c >= n || r >= n) return;
#pragma unroll
    for (int i = 0; i < BC; ++i)
        if (b0 + i < batch)
            Store<T>::store(x + (size_t)(b0 + i) * n * n + (size_t)r * n + c, acc[i] * scale_dt);
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

template <typename T, int BC>
static hipError_t launch_bp_tiled(const Geom &g, const BpWork &work, const void *y, void *x,
                                  int batch, float scale_dt, hipStream_t s) {
    constexpr int PLANES = BC / Chunk<T>::kImages;
    const int tiles = ((g.n + kBpTile - 1) / kBpTile) * ((g.n + kBpTile - 1) / kBpTile);
    dim3 grid(tiles, (batch + BC - 1) / BC);
    if (!g.fan) {
        const size_t lds = (size_t)PLANES * kBpAngles * work.window * sizeof(uint4);
        hipLaunchKernelGGL((bp_tiled_par<T, BC, 3, 3>), grid, dim3(256), lds, s, g, (const T *)y,
                           (T *)x, batch, scale_dt, work.window);
    } else {
        const size_t lds = (size_t)PLANES * kBpAnglesFan * work.window * sizeof(uint4) +
                           (size_t)kBpAnglesFan * work.window * sizeof(double4);
        if (work.bins <= 4)
            hipLaunchKernelGGL((bp_tiled_fan<T, BC, 4, 3>), grid, dim3(256), lds, s, g,
                               (const T *)y, (T *)x, batch, scale_dt, work.window);
        else
            hipLaunchKernelGGL((bp_tiled_fan<T, BC, 6, 3>), grid, dim3(256), lds, s, g,
                               (const T *)y, (T *)x, batch, scale_dt, work.window);
    }
    return hipGetLastError();
}

hipError_t launch_backproject(const Geom &g, const BpWork &work, int dtype, const LaunchShape &shape,
                              const void *y, void *x, int batch, float scale, hipStream_t s) {
    // every matrix entry carries the step length: R = step * (sum of sample weights)
    const float scale_dt = (float)(scale * g.step);
    if (shape.variant == VARIANT_TILED && work.window > 0) {
        switch (dtype) {
        case F32: return launch_bp_tiled<float, 32>(g, work, y, x, batch, scale_dt, s);
        case F16: return launch_bp_tiled<__half, 32>(g, work, y, x, batch, scale_dt, s);
        case BF16: return launch_bp_tiled<bf16_t, 32>(g, work, y, x, batch, scale_dt, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (dtype) {
    case F32: return launch_bp_direct<float, 4>(g, y, x, batch, scale_dt, s);
    case F16: return launch_bp_direct<__half, 4>(g, y, x, batch, scale_dt, s);
    case BF16: return launch_bp_direct<bf16_t, 4>(g, y, x, batch, scale_dt, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
