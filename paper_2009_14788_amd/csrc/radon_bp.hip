// Backprojection kernels: x[b][r][c] = scale * sum_{a,d} R[(a,d),(r,c)] * y[b][a][d].
//
// The exact transpose of the forward projection (TorchRadon uses it as the adjoint
// inside its CG solver, Sec. 4.3), computed as a gather: each thread owns pixels
// and collects, per angle, every sample of every ray whose bilinear footprint
// covers the pixel.  No atomics; results are deterministic.
#include "radon_common.hpp"
#include "radon_launch.hpp"
#include "radon_tiles.hpp"

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
// One block = one 16x16 pixel tile x BC images (blockIdx.y selects the images).
template <typename T, int BC, int NB, int NK, int AB>
__global__ __launch_bounds__(256) void bp_tiled_par(Geom g, const T *__restrict__ y,
                                                    T *__restrict__ x, int batch, float scale_dt,
                                                    int W) {
    extern __shared__ uint4 lds[];
    const ImageSet<T, BC> imgs = contiguous_images<T, BC>(
        y, (size_t)g.n_angles * g.det_count, x, (size_t)g.n * g.n, batch, blockIdx.y * BC, scale_dt);
    const SinoPointerSource<T, BC> src{imgs.in, g.det_count};
    bp_tile_par<T, BC, NB, NK, AB>(g, blockIdx.x, imgs, src, W, lds);
}

// Same, staging from the interleaved, zero-padded copy yi of the batch's sinograms
// (PAIRS: a copy of tap pairs, four images per chunk, applied with dot2), double-
// buffered with asynchronous copies (bp_tile_par_async).  Four resident blocks (four
// waves per SIMD) cap the registers at 128, so the plane pipeline of the inner loop
// does not lower the occupancy.
template <typename T, int BC, int NB, int NK, int AB, bool PAIRS = false>
__global__ __launch_bounds__(256, 4) void bp_tiled_par_il(Geom g, const uint4 *__restrict__ yi,
                                                       T *__restrict__ x, int batch, float scale_dt,
                                                       int W) {
    extern __shared__ uint4 lds[];
    constexpr int CH = PAIRS ? 4 : Chunk<T>::kImages;
    const int b0 = blockIdx.y * BC;
    // only the output side of the image set is used with an interleaved source
    const ImageSet<T, BC> imgs = contiguous_images<T, BC>(x, 0, x, (size_t)g.n * g.n, batch, b0, scale_dt);
    const int Dp = g.det_count + 2 * W;
    SinoInterleavedSource<T, BC, PAIRS> src;
    src.plane_stride = g.n_angles * Dp;
    src.base = yi + (size_t)(b0 / CH) * src.plane_stride;
    src.D = g.det_count;
    src.Dp = Dp;
    bp_tile_par_async<T, BC, NB, NK, AB, PAIRS>(g, blockIdx.x, imgs, src, W, lds);
}

template <typename T, int BC, int NB, int NK>
__global__ __launch_bounds__(256) void bp_tiled_fan(Geom g, const T *__restrict__ y,
                                                    T *__restrict__ x, int batch, float scale_dt,
                                                    int W) {
    extern __shared__ uint4 lds[];
    const ImageSet<T, BC> imgs = contiguous_images<T, BC>(
        y, (size_t)g.n_angles * g.det_count, x, (size_t)g.n * g.n, batch, blockIdx.y * BC, scale_dt);
    const SinoPointerSource<T, BC> src{imgs.in, g.det_count};
    bp_tile_fan<T, BC, NB, NK, kBpAnglesFan>(g, blockIdx.x, imgs, src, W, lds);
}

template <typename T, int BC, int NB, int NK, int AB, bool PAIRS = false>
__global__ __launch_bounds__(256) void bp_tiled_fan_il(Geom g, const uint4 *__restrict__ yi,
                                                       T *__restrict__ x, int batch, float scale_dt,
                                                       int W) {
    extern __shared__ uint4 lds[];
    constexpr int CH = PAIRS ? 4 : Chunk<T>::kImages;
    const int b0 = blockIdx.y * BC;
    const ImageSet<T, BC> imgs = contiguous_images<T, BC>(x, 0, x, (size_t)g.n * g.n, batch, b0, scale_dt);
    const int Dp = g.det_count + 2 * W;
    SinoInterleavedSource<T, BC, PAIRS> src;
    src.plane_stride = g.n_angles * Dp;
    src.base = yi + (size_t)(b0 / CH) * src.plane_stride;
    src.D = g.det_count;
    src.Dp = Dp;
    src.setup(W, AB * W);
    bp_tile_fan_async<T, BC, NB, NK, AB, PAIRS>(g, blockIdx.x, imgs, src, W, lds);
}

// Interleave sinograms y[B][A][D] into yi[groups][A][D + 2W] chunks of CH images with
// W zero bins on either side (images past B are zero).  Grid: (bins, A, groups).
template <typename T>
__global__ __launch_bounds__(256) void interleave_sinograms(const T *__restrict__ y, uint4 *__restrict__ yi,
                                                            int A, int D, int W, int batch) {
    constexpr int CH = Chunk<T>::kImages;
    const int Dp = D + 2 * W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= Dp) return;
    const int a = blockIdx.y, grp = blockIdx.z;
    const int d = p - W;
    const bool inside = (unsigned)d < (unsigned)D;
    T v[CH];
#pragma unroll
    for (int e = 0; e < CH; ++e) {
        const int b = grp * CH + e;
        v[e] = (inside && b < batch) ? y[((size_t)b * A + a) * D + d] : Chunk<T>::zero();
    }
    yi[((size_t)grp * A + a) * Dp + p] = Chunk<T>::pack(v);
}

// Tap-pair copy of 16-bit sinograms: chunk p of (grp, a) = bins d = p - W and d + 1
// of images 4 grp .. 4 grp + 3, one 32-bit word per image with bin d in the low half
// (zero outside the detector and past the batch).  Grid: (bins, A, groups).
template <typename T>
__global__ __launch_bounds__(256) void interleave_sino_pairs(const T *__restrict__ y, uint4 *__restrict__ yi,
                                                             int A, int D, int W, int batch) {
    constexpr int CH = Pair<T>::kImages;
    const int Dp = D + 2 * W;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= Dp) return;
    const int a = blockIdx.y, grp = blockIdx.z;
    const int d = p - W;
    const bool in0 = (unsigned)d < (unsigned)D, in1 = (unsigned)(d + 1) < (unsigned)D;
    uint32_t w[CH];
#pragma unroll
    for (int e = 0; e < CH; ++e) {
        const int b = grp * CH + e;
        const T *row = y + ((size_t)b * A + a) * D;
        const uint32_t lo = (in0 && b < batch) ? Pair<T>::bits(row[d]) : 0u;
        const uint32_t hi = (in1 && b < batch) ? Pair<T>::bits(row[d + 1]) : 0u;
        w[e] = lo | (hi << 16);
    }
    yi[((size_t)grp * A + a) * Dp + p] = make_uint4(w[0], w[1], w[2], w[3]);
}

// Workspace of the interleaved copies: four images per chunk (FP32, or 16-bit tap
// pairs; the 16-bit single-bin copies need half of it) in whole 64-image blocks.
size_t interleaved_sino_bytes(int n_angles, int det_count, int window, int batch, int /*dtype*/) {
    const size_t groups = ((size_t)batch + 63) / 64 * 64 / 4;
    return groups * (size_t)n_angles * (size_t)(det_count + 2 * window) * sizeof(uint4);
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

// Tiled backprojection from the tap-pair copy (16-bit storage, staging 2).  Returns
// false (nothing launched) when the window does not fit the staging slots.
// Angles per LDS block of the fan kernels on the interleaved copy: 2 when the shape
// asks for it, else kBpAnglesFan.
static int fan_block_angles(const LaunchShape &shape) { return shape.angles == 2 ? 2 : kBpAnglesFan; }

// Angles per LDS block of the parallel kernels on the interleaved copy (double-
// buffered): 2 when the shape asks for at most 2, else 4.
static int par_async_angles(const LaunchShape &shape) { return shape.angles <= 2 ? 2 : 4; }

// LDS of the double-buffered parallel kernels: two windows of ab angles, planes at the
// fixed pitch.
static size_t par_async_lds(int planes, int ab) { return 2 * (size_t)planes * ab * kBpWinPar * sizeof(uint4); }

// LDS of the double-buffered fan kernels: two sinogram windows and two FP32 ray windows
// of ab angles, and one window of raw FP64 rays.
static size_t fan_async_lds(int planes, int ab, int W) {
    return 2 * ((size_t)planes * ab * W * sizeof(uint4) + (size_t)ab * W * sizeof(float4)) +
           (size_t)ab * W * sizeof(double4);
}

template <typename T, int BC>
static bool launch_bp_pairs(const Geom &g, const BpWork &work, const LaunchShape &shape,
                            const void *y, void *x, int batch, float scale_dt, void *ws,
                            size_t ws_bytes, hipStream_t s, hipError_t *err) {
    constexpr int PLANES = BC / Pair<T>::kImages;
    const int W = work.window;
    const int dt = sizeof(T) == 4 ? F32 : F16;
    if (!(ws && ws_bytes >= interleaved_sino_bytes(g.n_angles, g.det_count, W, batch, dt) &&
          PLANES * W <= 256 * SinoInterleavedSource<T, BC, true>::kSlots &&
          (double)PLANES * g.n_angles * (g.det_count + 2.0 * W) < 2.0e9))
        return false;
    const int tiles = ((g.n + kBpTile - 1) / kBpTile) * ((g.n + kBpTile - 1) / kBpTile);
    dim3 grid(tiles, (batch + BC - 1) / BC);
    const int groups = (batch + BC - 1) / BC * PLANES;
    dim3 ig((g.det_count + 2 * W + 255) / 256, g.n_angles, groups);
    hipLaunchKernelGGL(interleave_sino_pairs<T>, ig, dim3(256), 0, s, (const T *)y, (uint4 *)ws,
                       g.n_angles, g.det_count, W, batch);
    *err = hipGetLastError();
    if (*err != hipSuccess) return true;
    const uint4 *yi = (const uint4 *)ws;
    if (!g.fan) {
        const int ab = par_async_angles(shape);
        const size_t lds = par_async_lds(PLANES, ab);
        if (ab == 2)
            hipLaunchKernelGGL((bp_tiled_par_il<T, BC, 3, 3, 2, true>), grid, dim3(256), lds, s, g, yi, (T *)x,
                               batch, scale_dt, W);
        else
            hipLaunchKernelGGL((bp_tiled_par_il<T, BC, 3, 3, 4, true>), grid, dim3(256), lds, s, g, yi, (T *)x,
                               batch, scale_dt, W);
    } else {
        const int ab = fan_block_angles(shape);
        const size_t lds = fan_async_lds(PLANES, ab, W);
        if (work.bins <= 4) {
            if (ab == 2)
                hipLaunchKernelGGL((bp_tiled_fan_il<T, BC, 4, 3, 2, true>), grid, dim3(256), lds, s, g, yi,
                                   (T *)x, batch, scale_dt, W);
            else
                hipLaunchKernelGGL((bp_tiled_fan_il<T, BC, 4, 3, kBpAnglesFan, true>), grid, dim3(256), lds,
                                   s, g, yi, (T *)x, batch, scale_dt, W);
        } else {
            if (ab == 2)
                hipLaunchKernelGGL((bp_tiled_fan_il<T, BC, 6, 3, 2, true>), grid, dim3(256), lds, s, g, yi,
                                   (T *)x, batch, scale_dt, W);
            else
                hipLaunchKernelGGL((bp_tiled_fan_il<T, BC, 6, 3, kBpAnglesFan, true>), grid, dim3(256), lds,
                                   s, g, yi, (T *)x, batch, scale_dt, W);
        }
    }
    *err = hipGetLastError();
    return true;
}

template <typename T, int BC>
static hipError_t launch_bp_tiled(const Geom &g, const BpWork &work, const LaunchShape &shape,
                                  const void *y, void *x, int batch, float scale_dt, void *ws,
                                  size_t ws_bytes, hipStream_t s) {
    constexpr int CH = Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    if constexpr (sizeof(T) == 2) {
        hipError_t err = hipSuccess;
        if (shape.stage == 2 &&
            launch_bp_pairs<T, BC>(g, work, shape, y, x, batch, scale_dt, ws, ws_bytes, s, &err))
            return err;
    }
    const int W = work.window;
    const int tiles = ((g.n + kBpTile - 1) / kBpTile) * ((g.n + kBpTile - 1) / kBpTile);
    dim3 grid(tiles, (batch + BC - 1) / BC);
    const int dt = sizeof(T) == 4 ? F32 : F16;
    const int groups = (batch + BC - 1) / BC * PLANES;
    // the interleaved copy: room in the workspace, slots for the window, 32-bit offsets
    const bool il = shape.stage && ws &&
                    ws_bytes >= interleaved_sino_bytes(g.n_angles, g.det_count, W, batch, dt) &&
                    PLANES * W <= 256 * SinoInterleavedSource<T, BC>::kSlots &&
                    (double)PLANES * g.n_angles * (g.det_count + 2.0 * W) < 2.0e9;
    if (il) {
        dim3 ig((g.det_count + 2 * W + 255) / 256, g.n_angles, groups);
        hipLaunchKernelGGL(interleave_sinograms<T>, ig, dim3(256), 0, s, (const T *)y, (uint4 *)ws,
                           g.n_angles, g.det_count, W, batch);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const uint4 *yi = (const uint4 *)ws;
    if (!g.fan) {
        if (il) {
            const int ab = par_async_angles(shape);
            const size_t lds = par_async_lds(PLANES, ab);
            if (ab == 2)
                hipLaunchKernelGGL((bp_tiled_par_il<T, BC, 3, 3, 2>), grid, dim3(256), lds, s, g, yi,
                                   (T *)x, batch, scale_dt, W);
            else
                hipLaunchKernelGGL((bp_tiled_par_il<T, BC, 3, 3, 4>), grid, dim3(256), lds, s, g, yi,
                                   (T *)x, batch, scale_dt, W);
        } else if (shape.angles <= 4) {
            const size_t lds = (size_t)PLANES * 4 * kBpWinPar * sizeof(uint4);
            hipLaunchKernelGGL((bp_tiled_par<T, BC, 3, 3, 4>), grid, dim3(256), lds, s, g,
                               (const T *)y, (T *)x, batch, scale_dt, W);
        } else {
            const size_t lds = (size_t)PLANES * kBpAngles * kBpWinPar * sizeof(uint4);
            hipLaunchKernelGGL((bp_tiled_par<T, BC, 3, 3, kBpAngles>), grid, dim3(256), lds, s, g,
                               (const T *)y, (T *)x, batch, scale_dt, W);
        }
    } else {
        // the caller's sinograms: kBpAnglesFan angles per block; the interleaved copy:
        // the shape's (2 or kBpAnglesFan)
        const int ab = il ? fan_block_angles(shape) : kBpAnglesFan;
        const size_t lds = il ? fan_async_lds(PLANES, ab, W)
                              : (size_t)PLANES * ab * W * sizeof(uint4) + (size_t)ab * W * sizeof(float4);
        if (work.bins <= 4) {
            if (il && ab == 2)
                hipLaunchKernelGGL((bp_tiled_fan_il<T, BC, 4, 3, 2>), grid, dim3(256), lds, s, g, yi,
                                   (T *)x, batch, scale_dt, W);
            else if (il)
                hipLaunchKernelGGL((bp_tiled_fan_il<T, BC, 4, 3, kBpAnglesFan>), grid, dim3(256), lds, s, g,
                                   yi, (T *)x, batch, scale_dt, W);
            else
                hipLaunchKernelGGL((bp_tiled_fan<T, BC, 4, 3>), grid, dim3(256), lds, s, g,
                                   (const T *)y, (T *)x, batch, scale_dt, W);
        } else {
            if (il && ab == 2)
                hipLaunchKernelGGL((bp_tiled_fan_il<T, BC, 6, 3, 2>), grid, dim3(256), lds, s, g, yi,
                                   (T *)x, batch, scale_dt, W);
            else if (il)
                hipLaunchKernelGGL((bp_tiled_fan_il<T, BC, 6, 3, kBpAnglesFan>), grid, dim3(256), lds, s, g,
                                   yi, (T *)x, batch, scale_dt, W);
            else
                hipLaunchKernelGGL((bp_tiled_fan<T, BC, 6, 3>), grid, dim3(256), lds, s, g,
                                   (const T *)y, (T *)x, batch, scale_dt, W);
        }
    }
    return hipGetLastError();
}

hipError_t launch_backproject(const Geom &g, const BpWork &work, int dtype, const LaunchShape &shape,
                              const void *y, void *x, int batch, float scale, void *ws,
                              size_t ws_bytes, hipStream_t s) {
    // every matrix entry carries the step length: R = step * (sum of sample weights)
    const float scale_dt = (float)(scale * g.step);
    if (shape.variant == VARIANT_TILED && work.window > 0) {
        const int im = shape.images;
#define RADON_BP_TILED(T, BC) launch_bp_tiled<T, BC>(g, work, shape, y, x, batch, scale_dt, ws, ws_bytes, s)
        // images per lane: 64, 32, 16, or one 16-byte chunk (4 FP32 / 8 16-bit images)
        switch (dtype) {
        case F32:
            return im >= 64 ? RADON_BP_TILED(float, 64)
                 : im >= 32 ? RADON_BP_TILED(float, 32)
                 : im >= 16 ? RADON_BP_TILED(float, 16) : RADON_BP_TILED(float, 4);
        case F16:
            return im >= 64 ? RADON_BP_TILED(__half, 64)
                 : im >= 32 ? RADON_BP_TILED(__half, 32)
                 : im >= 16 ? RADON_BP_TILED(__half, 16) : RADON_BP_TILED(__half, 8);
        case BF16:
            return im >= 64 ? RADON_BP_TILED(bf16_t, 64)
                 : im >= 32 ? RADON_BP_TILED(bf16_t, 32)
                 : im >= 16 ? RADON_BP_TILED(bf16_t, 16) : RADON_BP_TILED(bf16_t, 8);
        default: return hipErrorInvalidValue;
        }
#undef RADON_BP_TILED
    }
    switch (dtype) {
    case F32: return launch_bp_direct<float, 4>(g, y, x, batch, scale_dt, s);
    case F16: return launch_bp_direct<__half, 4>(g, y, x, batch, scale_dt, s);
    case BF16: return launch_bp_direct<bf16_t, 4>(g, y, x, batch, scale_dt, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
