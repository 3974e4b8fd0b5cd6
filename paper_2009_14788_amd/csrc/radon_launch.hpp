// Host-side launch interface between the C ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "radon_common.hpp"

namespace radon {

// Kernel families.
enum Variant { VARIANT_DIRECT = 0, VARIANT_TILED = 1 };

// Launch shape of one direction, chosen per plan (fixed default or autotuned).
struct LaunchShape {
    int variant = VARIANT_DIRECT;
    int images = 4;       // images per thread (accumulators per lane)
    int angles = 1;       // angles per block (forward: waves; backprojection: LDS angle block)
    int rays = 256;       // forward: bins per block; backprojection: pixels per block
    int stage = 1;        // tiled staging: 1 = interleaved workspace copy, 0 = caller's buffers,
                          // 2 = 16-bit tap-pair copy
    int tiling = 0;       // forward: index into kFwdTiling (slab rows, angles per item)
};

// ------------------------------------------------------------------ tiled forward work
// One work item of the tiled forward projector: up to W angles x up to 64
// consecutive bins (one lane per ray), marched through the image in slabs of
// H pixel rows (axis 0) or columns (axis 1), (H, W) the plan's tiling.  For every
// slab the item stages into LDS the pixel rows/columns [m_lo-1, m_lo+H+1] along the
// march axis and the transverse index range ranges[range + s - slab0] (inclusive,
// clamped to [-2, N+1]), where m_lo = -1 + s*H.
struct FwdItem {
    int a0, na;
    int d0, nd;
    int axis;
    int slab0, nslab;
    int range;
};

// Tilings of the tiled forward, chosen per plan by the autotuner: slab rows H, angles
// (waves of 64 lanes) per item W, and bins per 16-lane quarter wave Q (a quarter takes
// Q neighbouring bins x 16/Q neighbouring angles, so its taps fall on nearby columns).
// Tiling 0 (11-row slabs, 8 angles) keeps the FP32 8-image slab of a 512^2 item under
// 53 KB, so three 512-thread blocks share a compute unit's 160 KB of LDS; shorter
// slabs fit more blocks, longer ones stage fewer overlapping rows per sample, and
// 4-angle items suit few-angle geometries.
template <int H, int W, int Q>
struct FwdCfg {
    static constexpr int kSlabH = H;
    static constexpr int kWaves = W;
    static constexpr int kThreads = 64 * W;
    static constexpr int kQBins = Q;
    static constexpr int kQAngles = 16 / Q;
    static_assert(Q * kQAngles == 16 && W % kQAngles == 0, "lane mapping");
};
struct FwdTiling {
    int slab_h, waves, qbins;
};
constexpr int kFwdTilings = 4;
constexpr FwdTiling kFwdTiling[kFwdTilings] = {{11, 8, 2}, {7, 8, 2}, {15, 8, 2}, {11, 4, 4}};
using FwdCfg0 = FwdCfg<11, 8, 2>;
using FwdCfg1 = FwdCfg<7, 8, 2>;
using FwdCfg2 = FwdCfg<15, 8, 2>;
using FwdCfg3 = FwdCfg<11, 4, 4>;
// tiling 0, used by the uneven-batch kernels
constexpr int kSlabH = FwdCfg0::kSlabH;
constexpr int kFwdWaves = FwdCfg0::kWaves;
constexpr int kFwdThreads = FwdCfg0::kThreads;
#ifndef RADON_FWD_PITCH_MOD
#define RADON_FWD_PITCH_MOD 8
#endif
constexpr int kFwdPitchMod = RADON_FWD_PITCH_MOD; // LDS row pitch = 16k + this (chunks)
// Compile-time LDS row pitch (chunks, 16k + kFwdPitchMod) of the interleaved forward
// for plans whose windows all fit it (512^2 parallel plans need 118 columns); two
// planes of it leave room for three blocks in 160 KB.
constexpr int kFwdPitchFixed = 120;
static_assert(kFwdPitchFixed % 16 == kFwdPitchMod, "fixed pitch keeps the bank offset");
constexpr int kFwdLanes = 64;      // bins per forward item
constexpr int kTileTMax = 192;     // largest transverse extent of a staged slab

struct FwdWork {
    const FwdItem *items = nullptr;   // device
    const int2 *ranges = nullptr;     // device
    int n_items = 0;
    int tile_t = 0;                   // LDS row pitch in chunks (16k + 8, <= kTileTMax + 8)
};

// Host planning of the tiled forward projector from FP64 ray parameters
// (rays[a*D+d] = (ox, oy, sx, sy) in index coordinates) for slabs of slab_h rows and
// up to `angles` angles per item.  Returns false when some block of rays does not fit
// the tiled kernel; the direct kernel is used then.
bool plan_forward_tiles(int n, int n_angles, int det_count, const std::vector<double4> &rays,
                        int slab_h, int angles, std::vector<FwdItem> &items,
                        std::vector<int2> &ranges, int &tile_t);

// ws: optional workspace for the interleaved copy of the input batch (used by the
// tiled kernel when ws_bytes >= interleaved_bytes(n, batch, dtype)).
hipError_t launch_forward(const Geom &g, const FwdWork &work, int dtype, const LaunchShape &shape,
                          const void *x, void *y, int batch, float scale, void *ws,
                          size_t ws_bytes, hipStream_t s);
size_t interleaved_bytes(int n, int batch, int dtype);
// The tiled forward's interleaved copies of a batch (pairs: 16-bit tap pairs) into ws,
// `groups` groups of images (both orientations).
hipError_t launch_interleave(int dtype, bool pairs, const void *x, void *ws, int n, int batch,
                             int groups, hipStream_t s);
// Tiled forward of one tiling (radon_fwd_t<k>.hip); scale_dt = scale * step.
#define RADON_FWD_TILING_DECL(k)                                                                   \
    hipError_t launch_forward_tiling##k(const Geom &g, const FwdWork &work, int dtype,             \
                                        const LaunchShape &shape, const void *x, void *y, int batch, \
                                        float scale_dt, void *ws, size_t ws_bytes, hipStream_t s);
RADON_FWD_TILING_DECL(0)
RADON_FWD_TILING_DECL(1)
RADON_FWD_TILING_DECL(2)
RADON_FWD_TILING_DECL(3)
#undef RADON_FWD_TILING_DECL
// ------------------------------------------------------------------ tiled backprojection
constexpr int kBpTile = 16;        // pixels per tile side (one lane per pixel)
// angles per LDS block: from the caller's sinograms (parallel 8 or 4, fan 4); the
// double-buffered kernels on the interleaved copies take 4 or 2 (two windows in LDS)
constexpr int kBpAngles = 8;       // parallel beam, caller's sinograms
constexpr int kBpAnglesFan = 4;    // fan beam (rays are staged too)
// Parallel beam: LDS pitch (in chunks) of one staged angle's bin window.  The planner's
// window is 4 * ceil((floor(15 h / spacing) + 6) / 4) with h = |cos| + |sin| <= 1.5
// spacing (3 candidate bins must cover a footprint), so it never exceeds 28; a fixed
// pitch makes every plane offset of the LDS reads a compile-time immediate.
constexpr int kBpWinPar = 28;

struct BpWork {
    int window = 0;                // bins staged per (tile, angle); 0 = use the direct kernel
    int bins = 3;                  // candidate bins per (pixel, angle)
};

// Tiled backprojection plan: the bin window a 16x16 tile can touch at any angle and
// the number of candidate bins per pixel, such that the candidates (3 steps per bin)
// cover every sample within a pixel's footprint.  window = 0 when the tiled kernels
// do not apply (the direct kernel is used).
BpWork plan_backproject(int beam, int n, const std::vector<double2> &trig, double spacing,
                        double step, double source_distance, double det_distance);

// Backprojection of a batch (tiled kernels when the shape asks for them and work
// applies).  With shape.stage, a workspace ws of at least
// interleaved_sino_bytes(A, D, window, batch, dtype) bytes receives an interleaved,
// zero-padded copy of the sinograms first and the tiled kernel stages from it.
hipError_t launch_backproject(const Geom &g, const BpWork &work, int dtype, const LaunchShape &shape,
                              const void *y, void *x, int batch, float scale, void *ws,
                              size_t ws_bytes, hipStream_t s);
size_t interleaved_sino_bytes(int n_angles, int det_count, int window, int batch, int dtype);
hipError_t launch_dot_f64(const void *a, const void *b, long long n, int dtype, double *out,
                          double *partials, int n_partials, hipStream_t s);

// Per-system FP64 inner products of `batch` systems of n elements: out[b] = <a_b, b_b>.
// partials holds batch * dot_rows_chunks(n) doubles.  batch <= 65535.
constexpr int kDotRowChunks = 64;
int dot_rows_chunks(long long n);
hipError_t launch_dot_rows(const void *a, const void *b, long long n, int batch, int dtype,
                           double *out, double *partials, hipStream_t s);
// Fixed per-GPU partials of the no-allocation inner products: kStaticDotPartials
// doubles (512 KiB) in device memory that the library's code object holds until the
// process ends.  static_dot_partials returns the current device's address of it (looked
// up on the first call per device; no allocation).
constexpr int kStaticDotPartials = 1 << 16;
hipError_t static_dot_partials(double **out);
// out_b = u_b + c_b v_b with c_b = c0 * num[b] / den[b] in FP64 (null arrays read as 1,
// c_b = 0 where den[b] == 0, and then out_b = u_b without reading v).  batch <= 65535.
hipError_t launch_axpy_ratio(const void *u, const void *v, void *out, const double *num,
                             const double *den, double c0, long long n, int batch, int dtype,
                             hipStream_t s);
// p[0, n) = a reproducible pseudo-random pattern in [-0.5, 0.5) of type `dtype`.
hipError_t launch_fill_pattern(void *p, long long n, int dtype, unsigned seed, hipStream_t s);

}  // namespace radon
