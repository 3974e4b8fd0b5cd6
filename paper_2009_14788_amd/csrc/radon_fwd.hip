// Forward projection kernels: y[b][a][d] = scale * step * sum_k f_b(P_k(a, d)).
//
// Ray-driven (each line integral is sampled along the ray with bilinear
// interpolation and multiplied by the step length; TorchRadon Sec. 3.1.1-3.1.2,
// batch processing Sec. 4.1, FP32 arithmetic on 16-bit storage Sec. 3.3).
#include <algorithm>

#include "radon_common.hpp"
#include "radon_launch.hpp"
#include "radon_fwd_tiled.hpp"

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

// Interleaved copies of the call's images for the tiled kernels (tiling independent):
// `groups` groups of four images (tap pairs) or of Chunk<T>::kImages images.
hipError_t launch_interleave(int dtype, bool pairs, const void *x, void *ws, int n, int batch,
                             int groups, hipStream_t s) {
    const int tiles = (n + 4 + kIlTile - 1) / kIlTile;
    const dim3 grid(tiles * tiles, groups);
    switch (dtype * 2 + (pairs ? 1 : 0)) {
    case F32 * 2:
        hipLaunchKernelGGL(interleave_images<float>, grid, dim3(256), 0, s, (const float *)x, (uint4 *)ws,
                           n, batch, groups);
        break;
    case F16 * 2:
        hipLaunchKernelGGL(interleave_images<__half>, grid, dim3(256), 0, s, (const __half *)x, (uint4 *)ws,
                           n, batch, groups);
        break;
    case F16 * 2 + 1:
        hipLaunchKernelGGL(interleave_pairs<__half>, grid, dim3(256), 0, s, (const __half *)x, (uint4 *)ws,
                           n, batch, groups);
        break;
    case BF16 * 2:
        hipLaunchKernelGGL(interleave_images<bf16_t>, grid, dim3(256), 0, s, (const bf16_t *)x, (uint4 *)ws,
                           n, batch, groups);
        break;
    case BF16 * 2 + 1:
        hipLaunchKernelGGL(interleave_pairs<bf16_t>, grid, dim3(256), 0, s, (const bf16_t *)x, (uint4 *)ws,
                           n, batch, groups);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward(const Geom &g, const FwdWork &work, int dtype, const LaunchShape &shape,
                          const void *x, void *y, int batch, float scale, void *ws,
                          size_t ws_bytes, hipStream_t s) {
    const float scale_dt = (float)(scale * g.step);
    if (shape.variant == VARIANT_TILED && work.n_items > 0) {
        switch (shape.tiling) {
        case 0: return launch_forward_tiling0(g, work, dtype, shape, x, y, batch, scale_dt, ws, ws_bytes, s);
        case 1: return launch_forward_tiling1(g, work, dtype, shape, x, y, batch, scale_dt, ws, ws_bytes, s);
        case 2: return launch_forward_tiling2(g, work, dtype, shape, x, y, batch, scale_dt, ws, ws_bytes, s);
        case 3: return launch_forward_tiling3(g, work, dtype, shape, x, y, batch, scale_dt, ws, ws_bytes, s);
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
