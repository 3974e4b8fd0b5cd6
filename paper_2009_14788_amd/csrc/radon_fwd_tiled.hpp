// Tiled forward projection kernels (TorchRadon Sec. 3.1.1-3.1.2, batch processing
// Sec. 4.1, FP32 arithmetic on 16-bit storage Sec. 3.3), templated on the tiling C
// (slab rows, angles per item, lane mapping).  Each tiling is instantiated in a
// translation unit of its own (radon_fwd_t<k>.hip), so the kernels of the four
// tilings compile in parallel; radon_fwd.hip dispatches a call to the plan's tiling.
#pragma once

#include <type_traits>

#include "radon_common.hpp"
#include "radon_launch.hpp"
#include "radon_tiles.hpp"

namespace radon {

// Waves per SIMD that the LDS of one compute unit (160 KB, 4 SIMDs) holds for blocks
// of P planes at the fixed row pitch.
template <class C, int P>
constexpr int kFwdLdsWaves = (163840 / (P * (C::kSlabH + 3) * kFwdPitchFixed * 16)) * C::kWaves / 4;

// Waves per SIMD the tiled kernels are compiled for (it bounds their registers).
// Tiling 0: two-plane kernels (FP32 with 8 images, 16-bit with 16) are held to <= 80
// registers, so that LDS, not registers, caps them, at three blocks (6 waves per
// SIMD) for items up to ~120 columns wide; the FP32 kernel needs 66 registers then;
// the BF16 one spills one or two registers and still runs 12% faster than at two
// blocks.  Tap-pair kernels (16-bit, four images per chunk) have FP32's LDS
// footprint: the 8-image one is held to the same bound, the 16-image one fits one
// block per CU.  Other tilings: the waves their LDS allows, at most 6 (80 registers:
// the 16-image 16-bit kernels spill heavily at 64), none for one-plane kernels.
template <typename T, int BC, bool PAIRS, class C>
constexpr int fwd_min_waves() {
    if (std::is_same<C, FwdCfg0>::value)
        return PAIRS ? (BC == 8 ? 6 : 2) : ((sizeof(T) == 2 || BC == 8) ? 6 : 1);
    constexpr int P = BC / (PAIRS ? 4 : Chunk<T>::kImages);
    if (P == 1) return 1;
    constexpr int w = kFwdLdsWaves<C, (P > 1 ? P : 1)>;
    return w < 1 ? 1 : (w > 6 ? 6 : w);
}

// One block = one work item of the plan x BC images (blockIdx.y selects the images).
template <typename T, int BC, class C>
__global__ __launch_bounds__(C::kThreads, (fwd_min_waves<T, BC, false, C>())) void fwd_tiled(
    Geom g, FwdWork work, const T *__restrict__ x, T *__restrict__ y, int batch, float scale_dt,
    int tile_t) {
    extern __shared__ uint4 lds[];
    const FwdItem it = work.items[blockIdx.x];
    const ImageSet<T, BC> imgs = contiguous_images<T, BC>(
        x, (size_t)g.n * g.n, y, (size_t)g.n_angles * g.det_count, batch, blockIdx.y * BC, scale_dt);
    const PointerSource<T, BC, C> src{imgs.in, g.n};
    fwd_item<T, BC>(g, it, work.ranges, imgs, src, tile_t, lds);
}

// Same, staging from the interleaved, zero-bordered copies of the batch: xi holds
// the row-major copy [groups][N+4][N+4] followed by the transposed copy (PAIRS: copies
// of tap pairs, four images per chunk).  PITCH > 0: LDS rows of that many chunks (the
// plan's windows are at most that wide), fixed at compile time so the tap offsets are
// immediates.
template <typename T, int BC, int PITCH, bool PAIRS, class C>
__global__ __launch_bounds__(C::kThreads, (fwd_min_waves<T, BC, PAIRS, C>())) void fwd_tiled_il(
    Geom g, FwdWork work, const uint4 *__restrict__ xi, T *__restrict__ y, int batch, float scale_dt,
    int tile_t, int groups) {
    extern __shared__ uint4 lds[];
    constexpr int CH = PAIRS ? 4 : Chunk<T>::kImages;
    const FwdItem it = work.items[blockIdx.x];
    const int b0 = blockIdx.y * BC;
    // only the output side of the image set is used with an interleaved source
    const ImageSet<T, BC> imgs = contiguous_images<T, BC>(
        y, 0, y, (size_t)g.n_angles * g.det_count, batch, b0, scale_dt);
    const int plane = (g.n + 4) * (g.n + 4);
    const uint4 *first = xi + (size_t)(b0 / CH) * plane;
    const InterleavedSource<T, BC, PAIRS, C> src{first, first + (size_t)groups * plane, g.n, plane};
    fwd_item<T, BC, InterleavedSource<T, BC, PAIRS, C>, PITCH>(g, it, work.ranges, imgs, src, tile_t, lds);
}

// One storage type and lane width: stage 2 (16-bit) = tap-pair copy, 1 = interleaved
// copy, 0 = the caller's images (also when the workspace is missing or too small).
template <typename T, int BC, class C>
static hipError_t launch_fwd_tiled(const Geom &g, const FwdWork &work, const void *x, void *y,
                                   int batch, float scale_dt, int stage, void *ws, size_t ws_bytes,
                                   hipStream_t s) {
    constexpr int dt = std::is_same<T, float>::value ? F32 : (std::is_same<T, __half>::value ? F16 : BF16);
    const bool staged = ws && stage && ws_bytes >= interleaved_bytes(g.n, batch, dt);
    const bool pairs = sizeof(T) == 2 && stage == 2 && staged;
    const int ch = pairs ? 4 : Chunk<T>::kImages;
    const int planes = BC / ch;
    const size_t lds = (size_t)planes * (C::kSlabH + 3) * work.tile_t * sizeof(uint4);
    const size_t lds_fixed = (size_t)planes * (C::kSlabH + 3) * kFwdPitchFixed * sizeof(uint4);
    dim3 grid(work.n_items, (batch + BC - 1) / BC);
    if (!staged) {
        hipLaunchKernelGGL((fwd_tiled<T, BC, C>), grid, dim3(C::kThreads), lds, s, g, work, (const T *)x,
                           (T *)y, batch, scale_dt, work.tile_t);
        return hipGetLastError();
    }
    // groups of the launch: whole BC-image blocks (<= the groups interleaved_bytes counts)
    const int groups = (batch + BC - 1) / BC * planes;
    hipError_t e = launch_interleave(dt, pairs, x, ws, g.n, batch, groups, s);
    if (e != hipSuccess) return e;
    const bool fixed = work.tile_t <= kFwdPitchFixed;
    const uint4 *xi = (const uint4 *)ws;
    if constexpr (sizeof(T) == 2) {
        if (pairs) {
            if (fixed)
                hipLaunchKernelGGL((fwd_tiled_il<T, BC, kFwdPitchFixed, true, C>), grid, dim3(C::kThreads),
                                   lds_fixed, s, g, work, xi, (T *)y, batch, scale_dt, kFwdPitchFixed, groups);
            else
                hipLaunchKernelGGL((fwd_tiled_il<T, BC, 0, true, C>), grid, dim3(C::kThreads), lds, s, g,
                                   work, xi, (T *)y, batch, scale_dt, work.tile_t, groups);
            return hipGetLastError();
        }
    }
    if (fixed)
        hipLaunchKernelGGL((fwd_tiled_il<T, BC, kFwdPitchFixed, false, C>), grid, dim3(C::kThreads),
                           lds_fixed, s, g, work, xi, (T *)y, batch, scale_dt, kFwdPitchFixed, groups);
    else
        hipLaunchKernelGGL((fwd_tiled_il<T, BC, 0, false, C>), grid, dim3(C::kThreads), lds, s, g, work,
                           xi, (T *)y, batch, scale_dt, work.tile_t, groups);
    return hipGetLastError();
}

// All storage types and lane widths of tiling C (shape.images: FP32 4, 8 or 16, 16-bit
// 8 or 16 images per lane).
template <class C>
hipError_t launch_forward_tiled(const Geom &g, const FwdWork &work, int dtype, const LaunchShape &shape,
                                const void *x, void *y, int batch, float scale_dt, void *ws,
                                size_t ws_bytes, hipStream_t s) {
    const int st = shape.stage;
    switch (dtype) {
    case F32:
        if (shape.images <= 4)
            return launch_fwd_tiled<float, 4, C>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
        if (shape.images >= 16)
            return launch_fwd_tiled<float, 16, C>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
        return launch_fwd_tiled<float, 8, C>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
    case F16:
        if (shape.images >= 16)
            return launch_fwd_tiled<__half, 16, C>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
        return launch_fwd_tiled<__half, 8, C>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
    case BF16:
        if (shape.images >= 16)
            return launch_fwd_tiled<bf16_t, 16, C>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
        return launch_fwd_tiled<bf16_t, 8, C>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
