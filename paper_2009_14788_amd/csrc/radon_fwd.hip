// Forward projection kernels: y[b][a][d] = scale * step * sum_k f_b(P_k(a, d)).
//
// Ray-driven (each line integral is sampled along the ray with bilinear
// interpolation and multiplied by the step length; TorchRadon Sec. 3.1.1-3.1.2,
// batch processing Sec. 4.1, FP32 arithmetic on 16-bit storage Sec. 3.3).
#include "radon_common.hpp"
#include "radon_launch.hpp"

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
// Stage a rows x cols pixel window whose element (0, 0) is image pixel (ox0, oy0)
// into LDS as PLANES planes of 16-byte chunks (Chunk<T>::kImages images per chunk,
// zero outside the image).  Image base pointers are uniform per plane and image,
// so loads use 32-bit pixel offsets; the (row, col) walk is incremental.
template <typename T, int PLANES>
__device__ __forceinline__ void stage_window(uint4 *lds, int plane_chunks, int pitch,
                                             const T *const *img_base, int n, int ox0, int oy0,
                                             int rows, int cols) {
    constexpr int CH = Chunk<T>::kImages;
    const int total = rows * cols;
    const int step_i = 256 / cols, step_j = 256 - step_i * cols;
    int i0 = threadIdx.x / cols, j0 = threadIdx.x - (threadIdx.x / cols) * cols;
#pragma unroll
    for (int q = 0; q < PLANES; ++q) {
        int i = i0, jj = j0;
        for (int idx = threadIdx.x; idx < total; idx += 256) {
            const int gx = ox0 + jj, gy = oy0 + i;
            const bool inside = (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n;
            const unsigned off = inside ? (unsigned)(gy * n + gx) : 0u;
            T v[CH];
#pragma unroll
            for (int e = 0; e < CH; ++e) {
                const T val = img_base[q * CH + e][off];     // always a valid address
                v[e] = inside ? val : Chunk<T>::zero();
            }
            lds[q * plane_chunks + i * pitch + jj] = Chunk<T>::pack(v);
            jj += step_j;
            i += step_i;
            if (jj >= cols) {
                jj -= cols;
                ++i;
            }
        }
    }
}

// One block = one work item (up to 4 angles x 64 bins; wave w <-> angle a0+w, lane
// l <-> bin d0+l) x BC images.  The rays march through the image in slabs of
// kSlabH rows (or columns); per slab the block stages the slab's pixel window
// into LDS as 16-byte chunks holding Chunk<T>::kImages images each ("planes"),
// then every lane walks its ray's samples inside the slab.  A sample costs one
// address and weight computation shared by the BC images and four 16-byte LDS
// reads per plane.  The split of each ray's samples between slabs is fixed by
// FP64 boundary crossings (consistent across slabs); sample positions are FP64
// offsets from the lane's first cell in the slab and only the bilinear fractions
// drop to FP32, so weights are accurate to FP32 rounding anywhere in the image.
template <typename T, int BC>
__global__ __launch_bounds__(256) void fwd_tiled(Geom g, FwdWork work, const T *__restrict__ x,
                                                 T *__restrict__ y, int batch, float scale_dt,
                                                 int tile_t) {
    extern __shared__ uint4 lds[];
    constexpr int CH = Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    static_assert(BC % CH == 0, "BC must be a multiple of the images per chunk");
    const int plane_chunks = (kSlabH + 3) * tile_t;

    const FwdItem it = work.items[blockIdx.x];
    const int b0 = blockIdx.y * BC;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool active = wave < it.na && lane < it.nd;
    const int a = it.a0 + min(wave, it.na - 1), d = it.d0 + min(lane, it.nd - 1);
    const int n = g.n;
    const size_t img = (size_t)n * n;
    const T *img_base[BC];
#pragma unroll
    for (int e = 0; e < BC; ++e) img_base[e] = x + (size_t)min(b0 + e, batch - 1) * img;

    // the lane's ray, oriented so that the march coordinate grows with the sample index
    double4 r = ray_params(g, a, d);
    const double sm_raw = it.axis ? r.z : r.w;
    if (sm_raw < 0.0) { r.z = -r.z; r.w = -r.w; }
    const double om = it.axis ? r.x : r.y;
    const double inv_sm = 1.0 / fabs(sm_raw);
    int jlo, jhi;
    support_range(r, n, jlo, jhi);
    const int pitch = it.axis ? (kSlabH + 3) : tile_t;

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int si = 0; si < it.nslab; ++si) {
        const int2 tr = work.ranges[it.range + si];
        if (tr.x > tr.y) continue;                      // uniform over the block
        const int m_lo = -1 + (it.slab0 + si) * kSlabH;
        // tile element (0, 0) sits at image (ox0, oy0); tile is rows x cols pixels
        const int ox0 = it.axis ? m_lo - 1 : tr.x;
        const int oy0 = it.axis ? tr.x : m_lo - 1;
        const int cols = it.axis ? kSlabH + 3 : tr.y - tr.x + 1;
        const int rows = it.axis ? tr.y - tr.x + 1 : kSlabH + 3;

        __syncthreads();                                // previous slab fully consumed
        stage_window<T, PLANES>(lds, plane_chunks, pitch, img_base, n, ox0, oy0, rows, cols);
        __syncthreads();

        // samples of this ray whose march coordinate lies in [m_lo, m_lo + kSlabH)
        const int jb = max(jlo, (int)ceil(((double)m_lo - om) * inv_sm));
        const int je = min(jhi + 1, (int)ceil(((double)(m_lo + kSlabH) - om) * inv_sm));
        if (jb >= je) continue;
        const double px64 = fma((double)jb, r.z, r.x) - (double)ox0;
        const double py64 = fma((double)jb, r.w, r.y) - (double)oy0;
        const double bx = floor(px64), by = floor(py64);
        const double fxa = px64 - bx, fya = py64 - by;
        const int base = (int)by * pitch + (int)bx;
        const int max_addr = max((rows - 2) * pitch + (cols - 2), 0);
        // the slab's samples are summed separately and then added to the ray total
        // (two-level summation keeps FP32 rounding of long rays small)
        float part[BC];
#pragma unroll
        for (int i = 0; i < BC; ++i) part[i] = 0.0f;
        double jd = 0.0;
        for (int j = jb; j < je; ++j, jd += 1.0) {
            const double px = fma(jd, r.z, fxa), py = fma(jd, r.w, fya);
            const double cx = floor(px), cy = floor(py);
            const float fx = (float)(px - cx), fy = (float)(py - cy);
            const float gx = 1.0f - fx, gy = 1.0f - fy;
            const float w00 = __fmul_rn(gx, gy), w01 = __fmul_rn(fx, gy);
            const float w10 = __fmul_rn(gx, fy), w11 = __fmul_rn(fx, fy);
            int addr = base + __mul24((int)cy, pitch) + (int)cx;
            addr = min(max(addr, 0), max_addr);         // memory safety; real samples are inside
#pragma unroll
            for (int q = 0; q < PLANES; ++q) {
                const uint4 *pl = lds + q * plane_chunks + addr;
                const uint4 t00 = pl[0], t01 = pl[1], t10 = pl[pitch], t11 = pl[pitch + 1];
                float *aq = part + q * CH;
                Chunk<T>::fma(w00, t00, aq);
                Chunk<T>::fma(w01, t01, aq);
                Chunk<T>::fma(w10, t10, aq);
                Chunk<T>::fma(w11, t11, aq);
            }
        }
#pragma unroll
        for (int i = 0; i < BC; ++i) acc[i] += part[i];
    }
    if (!active) return;
#pragma unroll
    for (int i = 0; i < BC; ++i)
        if (b0 + i < batch)
            Store<T>::store(y + ((size_t)(b0 + i) * g.n_angles + a) * g.det_count + d,
                            acc[i] * scale_dt);
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

template <typename T, int BC>
static hipError_t launch_fwd_tiled(const Geom &g, const FwdWork &work, const void *x, void *y,
                                   int batch, float scale_dt, hipStream_t s) {
    constexpr int PLANES = BC / Chunk<T>::kImages;
    const size_t lds = (size_t)PLANES * (kSlabH + 3) * work.tile_t * sizeof(uint4);
    dim3 grid(work.n_items, (batch + BC - 1) / BC);
    hipLaunchKernelGGL((fwd_tiled<T, BC>), grid, dim3(256), lds, s, g, work, (const T *)x, (T *)y,
                       batch, scale_dt, work.tile_t);
    return hipGetLastError();
}

hipError_t launch_forward(const Geom &g, const FwdWork &work, int dtype, const LaunchShape &shape,
                          const void *x, void *y, int batch, float scale, hipStream_t s) {
    const float scale_dt = (float)(scale * g.step);
    if (shape.variant == VARIANT_TILED && work.n_items > 0) {
        const bool wide = shape.images >= 16;
        switch (dtype) {
        case F32:
            return wide ? launch_fwd_tiled<float, 16>(g, work, x, y, batch, scale_dt, s)
                        : launch_fwd_tiled<float, 8>(g, work, x, y, batch, scale_dt, s);
        case F16:
            return wide ? launch_fwd_tiled<__half, 16>(g, work, x, y, batch, scale_dt, s)
                        : launch_fwd_tiled<__half, 8>(g, work, x, y, batch, scale_dt, s);
        case BF16:
            return wide ? launch_fwd_tiled<bf16_t, 16>(g, work, x, y, batch, scale_dt, s)
                        : launch_fwd_tiled<bf16_t, 8>(g, work, x, y, batch, scale_dt, s);
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
