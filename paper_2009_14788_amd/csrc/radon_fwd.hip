// Forward projection kernels: y[b][a][d] = scale * step * sum_k f_b(P_k(a, d)).
//
// Ray-driven (each line integral is sampled along the ray with bilinear
// interpolation and multiplied by the step length; TorchRadon Sec. 3.1.1-3.1.2,
// batch processing Sec. 4.1, FP32 arithmetic on 16-bit storage Sec. 3.3).
#include <algorithm>

#include "radon_common.hpp"
#include "radon_launch.hpp"
#include "radon_tiles.hpp"

namespace radon {

// Direct variant: one thread per (ray, group of BC images); taps are read from
// global memory through the L1/L2 caches.  Serves every geometry and size.
template <typename T, int BC>
__global__ __launch_bounds__(256) void fwd_direct(Geom g, const T *__restrict__ x,
                                                  T *__restrict__ y, int batch, float scale_dt) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    const int b0 = blockIdx.z * BC;
    if (d >= g.det_count) return;
    const int n = g.n;
    const size_t img = (size_t)n * n;
    const double4 r = ray_params(g, a, d);
    int klo, khi;
    sample_range(r, n, klo, khi);

    const T *src[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) src[i] = x + (size_t)min(b0 + i, batch - 1) * img;

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int k = klo; k <= khi; ++k) {
        const double kd = (double)k;
        const Cell cx = cell_of(fma(kd, r.z, r.x)), cy = cell_of(fma(kd, r.w, r.y));
        const float wx0 = 1.0f - cx.f, wx1 = cx.f, wy0 = 1.0f - cy.f, wy1 = cy.f;
        const int c0 = cx.i, r0 = cy.i;
        const bool vc0 = (unsigned)c0 < (unsigned)n, vc1 = (unsigned)(c0 + 1) < (unsigned)n;
        const bool vr0 = (unsigned)r0 < (unsigned)n, vr1 = (unsigned)(r0 + 1) < (unsigned)n;
        const float w00 = (vr0 && vc0) ? __fmul_rn(wx0, wy0) : 0.0f;
        const float w01 = (vr0 && vc1) ? __fmul_rn(wx1, wy0) : 0.0f;
        const float w10 = (vr1 && vc0) ? __fmul_rn(wx0, wy1) : 0.0f;
        const float w11 = (vr1 && vc1) ? __fmul_rn(wx1, wy1) : 0.0f;
        // clamp addresses into the image; the weight of an outside tap is 0
        const int cc0 = min(max(c0, 0), n - 1), cc1 = min(max(c0 + 1, 0), n - 1);
        const int rr0 = min(max(r0, 0), n - 1), rr1 = min(max(r0 + 1, 0), n - 1);
        const size_t i00 = (size_t)rr0 * n + cc0, i01 = (size_t)rr0 * n + cc1;
        const size_t i10 = (size_t)rr1 * n + cc0, i11 = (size_t)rr1 * n + cc1;
#pragma unroll
        for (int i = 0; i < BC; ++i) {
            float v = acc[i];
            v = fmaf(w00, Store<T>::load(src[i] + i00), v);
            v = fmaf(w01, Store<T>::load(src[i] + i01), v);
            v = fmaf(w10, Store<T>::load(src[i] + i10), v);
            v = fmaf(w11, Store<T>::load(src[i] + i11), v);
            acc[i] = v;
        }
    }
#pragma unroll
    for (int i = 0; i < BC; ++i) {
        if (b0 + i < batch)
            Store<T>::store(y + ((size_t)(b0 + i) * g.n_angles + a) * g.det_count + d,
                            acc[i] * scale_dt);
    }
}

// ------------------------------------------------------------------ tiled variant
// Waves per SIMD the tiled kernels are compiled for: two-plane kernels (FP32 with 8
// images, 16-bit with 16) are held to <= 80 registers, so that LDS, not registers,
// caps them, at three blocks (6 waves per SIMD) for items up to ~120 columns wide.
// The FP32 kernel needs 66 registers then; the BF16 one spills one or two registers
// and still runs 12% faster than at two blocks.
// Tap-pair kernels (16-bit, four images per chunk) have FP32's LDS footprint: the
// 8-image one is held to the same bound; the 16-image one fits one block per CU.
template <typename T, int BC, bool PAIRS = false>
constexpr int kFwdMinWaves = PAIRS ? (BC == 8 ? 6 : 2) : ((sizeof(T) == 2 || BC == 8) ? 6 : 1);

// One block = one work item of the plan x BC images (blockIdx.y selects the images).
template <typename T, int BC>
__global__ __launch_bounds__(kFwdThreads, (kFwdMinWaves<T, BC>)) void fwd_tiled(Geom g, FwdWork work, const T *__restrict__ x,
                                                 T *__restrict__ y, int batch, float scale_dt,
                                                 int tile_t) {
    extern __shared__ uint4 lds[];
    const FwdItem it = work.items[blockIdx.x];
    const ImageSet<T, BC> imgs = contiguous_images<T, BC>(
        x, (size_t)g.n * g.n, y, (size_t)g.n_angles * g.det_count, batch, blockIdx.y * BC, scale_dt);
    const PointerSource<T, BC> src{imgs.in, g.n};
    fwd_item<T, BC>(g, it, work.ranges, imgs, src, tile_t, lds);
}

// Same, staging from the interleaved, zero-bordered copies of the batch: xi holds
// the row-major copy [groups][N+4][N+4] followed by the transposed copy (PAIRS: copies
// of tap pairs, four images per chunk).  PITCH > 0: LDS rows of that many chunks (the
// plan's windows are at most that wide), fixed at compile time so the tap offsets are
// immediates.
template <typename T, int BC, int PITCH, bool PAIRS = false>
__global__ __launch_bounds__(kFwdThreads, (kFwdMinWaves<T, BC, PAIRS>)) void fwd_tiled_il(Geom g, FwdWork work, const uint4 *__restrict__ xi,
                                                    T *__restrict__ y, int batch, float scale_dt,
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
    const InterleavedSource<T, BC, PAIRS> src{first, first + (size_t)groups * plane, g.n, plane};
    fwd_item<T, BC, InterleavedSource<T, BC, PAIRS>, PITCH>(g, it, work.ranges, imgs, src, tile_t, lds);
}

// Interleave a batch x[B][N][N] into chunks of CH images with a zero border of 2
// pixels (images past B are zero): xi[grp][y+2][x+2] (row-major copy) and
// xi[groups + grp][x+2][y+2] (transposed copy).  One block = one 16 x 16 chunk tile
// of one group, transposed through LDS so both stores are coalesced.
constexpr int kIlTile = 16;
template <typename T>
__global__ __launch_bounds__(256) void interleave_images(const T *__restrict__ x, uint4 *__restrict__ xi,
                                                         int n, int batch, int groups) {
    constexpr int CH = Chunk<T>::kImages;
    __shared__ uint4 tile[kIlTile][kIlTile + 1];
    const int np = n + 4;
    const int tiles = (np + kIlTile - 1) / kIlTile;
    const int grp = blockIdx.y;
    const int ty0 = (blockIdx.x / tiles) * kIlTile, tx0 = (blockIdx.x % tiles) * kIlTile;
    const int tx = threadIdx.x % kIlTile, ty = threadIdx.x / kIlTile;
    const size_t plane = (size_t)np * np;
    {   // padded row-major coordinates (xx, yy) of this thread's chunk
        const int xx = tx0 + tx, yy = ty0 + ty;
        const int ix = xx - 2, iy = yy - 2;
        const bool inside = (unsigned)ix < (unsigned)n && (unsigned)iy < (unsigned)n;
        T v[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int b = grp * CH + e;
            v[e] = (inside && b < batch) ? x[(size_t)b * n * n + (size_t)iy * n + ix] : Chunk<T>::zero();
        }
        const uint4 c = Chunk<T>::pack(v);
        tile[ty][tx] = c;
        if (xx < np && yy < np) xi[(size_t)grp * plane + (size_t)yy * np + xx] = c;
    }
    __syncthreads();
    {   // transposed copy: row = padded x, column = padded y
        const int row = tx0 + ty, col = ty0 + tx;
        if (row < np && col < np)
            xi[(size_t)(groups + grp) * plane + (size_t)row * np + col] = tile[tx][ty];
    }
}

// Tap-pair copies of a 16-bit batch: the same chunk grid as interleave_images, chunk
// (grp, yy, xx) = padded pixels xx and xx + 1 of padded row yy (row-major copy) and
// chunk (groups + grp, xx, yy) = padded pixels (xx, yy) and (xx, yy + 1) (transposed
// copy: pairs run along the image's y), word e of a chunk = image 4 grp + e with the
// first pixel in its low half.  One block = one 16 x 16 chunk tile of one group, read
// with one pixel of halo into LDS.
template <typename T>
__global__ __launch_bounds__(256) void interleave_pairs(const T *__restrict__ x, uint4 *__restrict__ xi,
                                                        int n, int batch, int groups) {
    constexpr int CH = Pair<T>::kImages;
    constexpr int TP = kIlTile + 1;
    __shared__ uint2 tile[TP][TP + 1];   // 4 images' 16-bit values per padded pixel
    const int np = n + 4;
    const int tiles = (np + kIlTile - 1) / kIlTile;
    const int grp = blockIdx.y;
    const int ty0 = (blockIdx.x / tiles) * kIlTile, tx0 = (blockIdx.x % tiles) * kIlTile;
    const size_t plane = (size_t)np * np;
    for (int t = threadIdx.x; t < TP * TP; t += 256) {
        const int i = t / TP, j = t - i * TP;
        const int ix = tx0 + j - 2, iy = ty0 + i - 2;
        const bool inside = (unsigned)ix < (unsigned)n && (unsigned)iy < (unsigned)n;
        uint32_t h[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int b = grp * CH + e;
            h[e] = (inside && b < batch) ? Pair<T>::bits(x[(size_t)b * n * n + (size_t)iy * n + ix]) : 0u;
        }
        tile[i][j] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
    __syncthreads();
    // pixels a (low halves) and b (high halves) of the four images
    auto pair = [](uint2 a, uint2 b) {
        return make_uint4((a.x & 0xffffu) | (b.x << 16), (a.x >> 16) | (b.x & 0xffff0000u),
                          (a.y & 0xffffu) | (b.y << 16), (a.y >> 16) | (b.y & 0xffff0000u));
    };
    const int tx = threadIdx.x % kIlTile, ty = threadIdx.x / kIlTile;
    {
        const int xx = tx0 + tx, yy = ty0 + ty;
        if (xx < np && yy < np) xi[(size_t)grp * plane + (size_t)yy * np + xx] = pair(tile[ty][tx], tile[ty][tx + 1]);
    }
    {
        const int row = tx0 + ty, col = ty0 + tx;   // padded x, padded y
        if (row < np && col < np)
            xi[(size_t)(groups + grp) * plane + (size_t)row * np + col] = pair(tile[tx][ty], tile[tx + 1][ty]);
    }
}

// Workspace of the interleaved copies: four images per chunk (FP32, or 16-bit tap
// pairs; the 16-bit single-pixel copies need half of it) in whole 16-image blocks.
size_t interleaved_bytes(int n, int batch, int /*dtype*/) {
    const size_t groups = ((size_t)batch + 15) / 16 * 16 / 4;
    return 2 * groups * (size_t)(n + 4) * (n + 4) * sizeof(uint4);
}

template <typename T, int BC>
static hipError_t launch_fwd_direct(const Geom &g, const void *x, void *y, int batch,
                                    float scale_dt, hipStream_t s) {
    dim3 block(256);
    dim3 grid((g.det_count + 255) / 256, g.n_angles, (batch + BC - 1) / BC);
    hipLaunchKernelGGL((fwd_direct<T, BC>), grid, block, 0, s, g, (const T *)x, (T *)y, batch,
                       scale_dt);
    return hipGetLastError();
}

// Tiled forward with 16-bit tap pairs (stage 2): pair copies, then the pair kernel.
template <typename T, int BC>
static hipError_t launch_fwd_pairs(const Geom &g, const FwdWork &work, const void *x, void *y,
                                   int batch, float scale_dt, void *ws, hipStream_t s) {
    constexpr int PLANES = BC / Pair<T>::kImages;
    const size_t lds = (size_t)PLANES * (kSlabH + 3) * work.tile_t * sizeof(uint4);
    const size_t lds_fixed = (size_t)PLANES * (kSlabH + 3) * kFwdPitchFixed * sizeof(uint4);
    dim3 grid(work.n_items, (batch + BC - 1) / BC);
    const int groups = (batch + BC - 1) / BC * PLANES;
    const int tiles = (g.n + 4 + kIlTile - 1) / kIlTile;
    hipLaunchKernelGGL(interleave_pairs<T>, dim3(tiles * tiles, groups), dim3(256), 0, s,
                       (const T *)x, (uint4 *)ws, g.n, batch, groups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (work.tile_t <= kFwdPitchFixed)
        hipLaunchKernelGGL((fwd_tiled_il<T, BC, kFwdPitchFixed, true>), grid, dim3(kFwdThreads),
                           lds_fixed, s, g, work, (const uint4 *)ws, (T *)y, batch, scale_dt,
                           kFwdPitchFixed, groups);
    else
        hipLaunchKernelGGL((fwd_tiled_il<T, BC, 0, true>), grid, dim3(kFwdThreads), lds, s, g, work,
                           (const uint4 *)ws, (T *)y, batch, scale_dt, work.tile_t, groups);
    return hipGetLastError();
}

template <typename T, int BC>
static hipError_t launch_fwd_tiled(const Geom &g, const FwdWork &work, const void *x, void *y,
                                   int batch, float scale_dt, int stage, void *ws, size_t ws_bytes,
                                   hipStream_t s) {
    constexpr int CH = Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    const size_t lds = (size_t)PLANES * (kSlabH + 3) * work.tile_t * sizeof(uint4);
    const size_t lds_fixed = (size_t)PLANES * (kSlabH + 3) * kFwdPitchFixed * sizeof(uint4);
    dim3 grid(work.n_items, (batch + BC - 1) / BC);
    const int dt = sizeof(T) == 4 ? F32 : F16;
    if constexpr (sizeof(T) == 2) {
        if (stage == 2 && ws && ws_bytes >= interleaved_bytes(g.n, batch, dt))
            return launch_fwd_pairs<T, BC>(g, work, x, y, batch, scale_dt, ws, s);
    }
    if (ws && stage && ws_bytes >= interleaved_bytes(g.n, batch, dt)) {
        // groups of the launch: whole BC-image blocks (<= the groups interleaved_bytes counts)
        const int groups = (batch + BC - 1) / BC * PLANES;
        const int tiles = (g.n + 4 + kIlTile - 1) / kIlTile;
        hipLaunchKernelGGL(interleave_images<T>, dim3(tiles * tiles, groups), dim3(256), 0, s,
                           (const T *)x, (uint4 *)ws, g.n, batch, groups);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (work.tile_t <= kFwdPitchFixed)
            hipLaunchKernelGGL((fwd_tiled_il<T, BC, kFwdPitchFixed>), grid, dim3(kFwdThreads),
                               lds_fixed, s, g, work, (const uint4 *)ws, (T *)y, batch, scale_dt,
                               kFwdPitchFixed, groups);
        else
            hipLaunchKernelGGL((fwd_tiled_il<T, BC, 0>), grid, dim3(kFwdThreads), lds, s, g, work,
                               (const uint4 *)ws, (T *)y, batch, scale_dt, work.tile_t, groups);
    } else {
        hipLaunchKernelGGL((fwd_tiled<T, BC>), grid, dim3(kFwdThreads), lds, s, g, work, (const T *)x,
                           (T *)y, batch, scale_dt, work.tile_t);
    }
    return hipGetLastError();
}

hipError_t launch_forward(const Geom &g, const FwdWork &work, int dtype, const LaunchShape &shape,
                          const void *x, void *y, int batch, float scale, void *ws,
                          size_t ws_bytes, hipStream_t s) {
    const float scale_dt = (float)(scale * g.step);
    if (shape.variant == VARIANT_TILED && work.n_items > 0) {
        const int st = shape.stage;
        switch (dtype) {
        case F32:
            if (shape.images <= 4)
                return launch_fwd_tiled<float, 4>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
            return launch_fwd_tiled<float, 8>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
        case F16:
            if (shape.images >= 16)
                return launch_fwd_tiled<__half, 16>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
            return launch_fwd_tiled<__half, 8>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
        case BF16:
            if (shape.images >= 16)
                return launch_fwd_tiled<bf16_t, 16>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
            return launch_fwd_tiled<bf16_t, 8>(g, work, x, y, batch, scale_dt, st, ws, ws_bytes, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (dtype) {
    case F32: return launch_fwd_direct<float, 4>(g, x, y, batch, scale_dt, s);
    case F16: return launch_fwd_direct<__half, 4>(g, x, y, batch, scale_dt, s);
    case BF16: return launch_fwd_direct<bf16_t, 4>(g, x, y, batch, scale_dt, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace radon
