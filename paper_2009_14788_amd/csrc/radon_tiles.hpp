// Per-work-item device functions of the tiled projectors, shared by the per-call
// kernels and the persistent uneven-batch kernels.  Every function is called by all
// threads of a block (the tiling's C::kThreads for the forward, 256 for the
// backprojection) with block-uniform arguments (they contain barriers).
#pragma once

#include "radon_common.hpp"
#include "radon_launch.hpp"
#include "radon_lds_dma.hpp"

namespace radon {

// The BC images one block works on: input and output base pointers (entries past
// `count` repeat a valid input so loads stay in bounds; their outputs are never
// written) and the per-image output scale (scale * step).
template <typename T, int BC>
struct ImageSet {
    const T *in[BC];
    T *out[BC];
    float scale[BC];
    int count;
};

// Images b0 .. b0+BC-1 of one contiguous batch (input stride `in_stride`, output
// stride `out_stride` elements).
template <typename T, int BC>
__device__ __forceinline__ ImageSet<T, BC> contiguous_images(const T *in, size_t in_stride, T *out,
                                                             size_t out_stride, int batch, int b0,
                                                             float scale_dt) {
    ImageSet<T, BC> s;
#pragma unroll
    for (int e = 0; e < BC; ++e) {
        const int b = min(b0 + e, batch - 1);
        s.in[e] = in + (size_t)b * in_stride;
        s.out[e] = out + (size_t)b * out_stride;
        s.scale[e] = scale_dt;
    }
    s.count = min(BC, batch - b0);
    return s;
}

// ------------------------------------------------------------------ forward
// Slab staging sources.  Both fill a rows x cols pixel window of the staging frame
// whose element (0, 0) is frame pixel (ox0, oy0) into LDS as PLANES planes of 16-byte
// chunks (Chunk<T>::kImages images per chunk, zero outside the image), rows `pitch`
// chunks apart and planes `plane_chunks` apart.  A source with kMarchFrame stages in
// the march frame: for items that march along x (axis 1) the frame is the transposed
// image, so every slab is a band of rows; otherwise the frame is the image.  Cfg: the
// forward tiling (block size, slab rows) the source serves.

// From the callers' images (any layout of BC image pointers), in the image frame:
// image base pointers are uniform per plane and image, loads use 32-bit pixel
// offsets, the (row, col) walk is incremental, and pixels outside the image read a
// valid address and are replaced by 0.
template <typename T, int BC, class C = FwdCfg0>
struct PointerSource {
    using Cfg = C;
    static constexpr bool kMarchFrame = false;
    static constexpr bool kPairs = false;
    const T *const *img;
    int n;
    __device__ __forceinline__ void stage(uint4 *lds, int plane_chunks, int pitch, int ox0, int oy0,
                                          int rows, int cols, int /*axis*/) const {
        constexpr int CH = Chunk<T>::kImages;
        constexpr int PLANES = BC / CH;
        const int total = rows * cols;
        const int step_i = C::kThreads / cols, step_j = C::kThreads - step_i * cols;
        const int i0 = threadIdx.x / cols, j0 = threadIdx.x - i0 * cols;
#pragma unroll
        for (int q = 0; q < PLANES; ++q) {
            int i = i0, jj = j0;
            for (int idx = threadIdx.x; idx < total; idx += C::kThreads) {
                const int gx = ox0 + jj, gy = oy0 + i;
                const bool inside = (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n;
                const unsigned off = inside ? (unsigned)(gy * n + gx) : 0u;
                T v[CH];
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    const T val = img[q * CH + e][off];     // always a valid address
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
};

// From the callers' 16-bit images as tap pairs (Pair<T>, four images per chunk), in the
// image frame: chunk (row, col) holds, in word e, pixels col and col + 1 of that row
// of image e (the first in the low half), so that one 16-byte read per row serves a
// sample's two horizontal taps of four images.  The walk is PointerSource's.  For an
// even image side and 4-byte aligned images (the usual case) a thread reads the 32-bit
// words w(g) = pixels (2g, 2g + 1) and w(g + 1) of each image and forms the chunks at
// columns 2g (w(g) itself) and 2g + 1 (high half of w(g), low half of w(g + 1)): one
// 32-bit load per chunk and image instead of two 16-bit ones; a word is then either
// wholly inside the row or wholly outside it.
template <typename T, class C = FwdCfg0>
struct PairPointerSource {
    using Cfg = C;
    static constexpr bool kMarchFrame = false;
    static constexpr bool kPairs = true;
    const T *const *img;   // four image base pointers
    int n;
    __device__ __forceinline__ void stage(uint4 *lds, int /*plane_chunks*/, int pitch, int ox0, int oy0,
                                          int rows, int cols, int /*axis*/) const {
        bool words = (n & 1) == 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) words = words && ((uintptr_t)img[e] & 3u) == 0;
        if (words)
            stage_words(lds, pitch, ox0, oy0, rows, cols);
        else
            stage_pixels(lds, pitch, ox0, oy0, rows, cols);
    }

    __device__ __forceinline__ void stage_words(uint4 *lds, int pitch, int ox0, int oy0, int rows,
                                                int cols) const {
        const int hn = n >> 1;                          // words per image row
        const int g0 = ox0 >> 1;                        // floor: ox0 >= -2
        const int wcols = ((ox0 + cols - 1) >> 1) - g0 + 1;
        const int total = rows * wcols;
        const int step_i = C::kThreads / wcols, step_j = C::kThreads - step_i * wcols;
        int i = threadIdx.x / wcols, jj = threadIdx.x - i * wcols;
        for (int idx = threadIdx.x; idx < total; idx += C::kThreads) {
            const int g = g0 + jj, gy = oy0 + i;
            const bool row_in = (unsigned)gy < (unsigned)n;
            const bool in0 = row_in && (unsigned)g < (unsigned)hn;
            const bool in1 = row_in && (unsigned)(g + 1) < (unsigned)hn;
            const unsigned off0 = in0 ? (unsigned)(gy * hn + g) : 0u;
            const unsigned off1 = in1 ? (unsigned)(gy * hn + g + 1) : 0u;
            uint32_t a[4], b[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t *row = reinterpret_cast<const uint32_t *>(img[e]);
                const uint32_t wa = row[off0], wb = row[off1];  // always valid addresses
                a[e] = in0 ? wa : 0u;
                b[e] = in1 ? wb : 0u;
            }
            const int c0 = 2 * g - ox0;                     // chunk columns c0 and c0 + 1
            if (c0 >= 0 && c0 < cols) lds[i * pitch + c0] = make_uint4(a[0], a[1], a[2], a[3]);
            if (c0 + 1 >= 0 && c0 + 1 < cols)
                lds[i * pitch + c0 + 1] =
                    make_uint4((a[0] >> 16) | (b[0] << 16), (a[1] >> 16) | (b[1] << 16),
                               (a[2] >> 16) | (b[2] << 16), (a[3] >> 16) | (b[3] << 16));
            jj += step_j;
            i += step_i;
            if (jj >= wcols) {
                jj -= wcols;
                ++i;
            }
        }
    }

    __device__ __forceinline__ void stage_pixels(uint4 *lds, int pitch, int ox0, int oy0, int rows,
                                                 int cols) const {
        const int total = rows * cols;
        const int step_i = C::kThreads / cols, step_j = C::kThreads - step_i * cols;
        int i = threadIdx.x / cols, jj = threadIdx.x - i * cols;
        for (int idx = threadIdx.x; idx < total; idx += C::kThreads) {
            const int gx = ox0 + jj, gy = oy0 + i;
            const bool row_in = (unsigned)gy < (unsigned)n;
            const bool in0 = row_in && (unsigned)gx < (unsigned)n;
            const bool in1 = row_in && (unsigned)(gx + 1) < (unsigned)n;
            const unsigned off0 = in0 ? (unsigned)(gy * n + gx) : 0u;
            const unsigned off1 = in1 ? (unsigned)(gy * n + gx + 1) : 0u;
            uint32_t w[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t lo = Pair<T>::bits(img[e][off0]);     // always valid addresses
                const uint32_t hi = Pair<T>::bits(img[e][off1]);
                w[e] = (in0 ? lo : 0u) | ((in1 ? hi : 0u) << 16);
            }
            lds[i * pitch + jj] = make_uint4(w[0], w[1], w[2], w[3]);
            jj += step_j;
            i += step_i;
            if (jj >= cols) {
                jj -= cols;
                ++i;
            }
        }
    }
};

// From the interleaved copies of the batch, in the march frame: chunk (group, y+2,
// x+2) of the row-major copy [groups][N+4][N+4] holds pixel (x, y) of the group's
// images, and chunk (group, x+2, y+2) of the transposed copy holds the same pixel,
// both with a zero border of 2 pixels, so a window inside [-2, N+1]^2 is copied chunk
// for chunk with no bounds test.  PAIRS (16-bit storage): the copies hold tap pairs
// (Pair<T>) instead, chunk (group, row, col) = frame pixels col and col + 1 of the row,
// four images per chunk.  Window rows/columns beyond [-2, N+1] are never
// tapped and are not staged.  Wave w copies window rows w, w+W, w+2W, ... (W waves; a
// slab has H + 3 rows) with its lanes along the row (at most kTileTMax = 3 x 64
// chunks), from wave-uniform row addresses.
template <typename T, int BC, bool PAIRS = false, class C = FwdCfg0>
struct InterleavedSource {
    using Cfg = C;
    static constexpr bool kMarchFrame = true;
    static constexpr bool kPairs = PAIRS;
    const uint4 *base;   // row-major copy: first plane of the block's images
    const uint4 *tbase;  // transposed copy: first plane of the block's images
    int n;
    int plane_stride;    // chunks between planes ((N+4)^2)
    __device__ __forceinline__ void stage(uint4 *lds, int plane_chunks, int pitch, int ox0, int oy0,
                                          int rows, int cols, int axis) const {
        static_assert(kTileTMax <= 3 * 64, "staging loop bounds");
        constexpr int kRowsPerWave = (C::kSlabH + 3 + C::kWaves - 1) / C::kWaves;
        constexpr int PLANES = BC / (PAIRS ? 4 : Chunk<T>::kImages);
        const int np = n + 4;
        const int r_end = min(rows, n + 2 - oy0), c_end = min(cols, n + 2 - ox0);
        if (r_end <= 0 || c_end <= 0) return;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        const uint4 *src0 = (axis ? tbase : base) + (oy0 + 2) * np + (ox0 + 2);
        // every window row of every plane goes straight from global memory into LDS
        // (lds_copy16_async: a wave's 64 lanes fill 64 consecutive chunks of the row),
        // all in flight together, then one wait: one global round trip per slab instead
        // of one per row.  Row and column-block tests are wave-uniform; lanes past the
        // window end are masked off.
#pragma unroll
        for (int q = 0; q < PLANES; ++q) {
            const uint4 *src = src0 + q * plane_stride;
            uint4 *dst = lds + q * plane_chunks;
#pragma unroll
            for (int i = 0; i < kRowsPerWave; ++i) {
                const int row = wave + C::kWaves * i;
                if (row >= r_end) break;
                const uint4 *srow = src + row * np;
                uint4 *drow = dst + row * pitch;
                if (lane < c_end) lds_copy16_async(srow + lane, drow);
                if (c_end > 64 && lane + 64 < c_end) lds_copy16_async(srow + lane + 64, drow + 64);
                if (c_end > 128 && lane + 128 < c_end) lds_copy16_async(srow + lane + 128, drow + 128);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);     // this wave's copies have landed (the caller's
                                           // barrier publishes everyone's)
    }
};

// The samples of one lane's ray inside one slab: `cnt` samples at frame offsets
// (fxa + j sx, fya + j sy) >= 1 from the lane's anchor chunk, stepped in FP32: the
// offsets stay below ~20 pixels, so a position carries at most ~2e-6 pixel of
// rounding (FP32 image coordinates would carry 3e-5 at the edge of a 512^2 image),
// and the two FP64 conversions per sample are saved.  SWAP: the frame is the
// transposed image; the two middle taps are then taken in the image frame's order,
// so both frames give bitwise identical sums.  PITCH > 0: the row pitch is that
// compile-time number of chunks (planes of SH + 3 rows), so every tap offset is an
// immediate of the LDS read instead of a per-sample address add.
template <typename T, int BC, bool SWAP, int PITCH, int SH>
__device__ __forceinline__ void slab_samples(const uint4 *lane_lds, int pitch, int plane_chunks,
                                             double fxa, double fya, double sx, double sy, int cnt,
                                             float *part) {
    constexpr int CH = Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    if (PITCH > 0) {
        pitch = PITCH;
        plane_chunks = (SH + 3) * PITCH;
    }
    // byte addressing: one multiply-add and one shift-add per sample, the tap
    // offsets (+16 bytes, +pitch, +plane) are loop invariants
    const char *base = reinterpret_cast<const char *>(lane_lds);
    const unsigned row_bytes = (unsigned)pitch * 16u, plane_bytes = (unsigned)plane_chunks * 16u;
    const float end = (float)cnt, fxa32 = (float)fxa, fya32 = (float)fya;
    const float sx32 = (float)sx, sy32 = (float)sy;
    for (float jf = 0.0f; jf < end; jf += 1.0f) {
        const float px = fmaf(jf, sx32, fxa32), py = fmaf(jf, sy32, fya32);
        const int cx = (int)px, cy = (int)py;                       // px, py >= 1 - 1e-6
        const float fx = __builtin_amdgcn_fractf(px), fy = __builtin_amdgcn_fractf(py);
        // bilinear weights in the image frame (a, b: the image's x and y fractions), two
        // of them as differences: five VALU instructions instead of six
        const float a = SWAP ? fy : fx, b = SWAP ? fx : fy;
        const float gb = 1.0f - b;
        const float i01 = __fmul_rn(a, gb), i11 = __fmul_rn(a, b);
        const float i00 = gb - i01, i10 = b - i11;
        // frame taps: with SWAP the frame's x + 1 neighbour is the image's y + 1
        const float w00 = i00, w11 = i11, w01 = SWAP ? i10 : i01, w10 = SWAP ? i01 : i10;
        const char *p0 = base + ((unsigned)__mul24(cy, pitch) + (unsigned)cx) * 16u;
#pragma unroll
        for (int q = 0; q < PLANES; ++q) {
            const char *pq = p0 + q * plane_bytes;
            const uint4 t00 = *reinterpret_cast<const uint4 *>(pq);
            const uint4 t01 = *reinterpret_cast<const uint4 *>(pq + 16);
            const uint4 t10 = *reinterpret_cast<const uint4 *>(pq + row_bytes);
            const uint4 t11 = *reinterpret_cast<const uint4 *>(pq + row_bytes + 16);
            float *aq = part + q * CH;
            Chunk<T>::fma(w00, t00, aq);
            if (SWAP) {
                Chunk<T>::fma(w10, t10, aq);
                Chunk<T>::fma(w01, t01, aq);
            } else {
                Chunk<T>::fma(w01, t01, aq);
                Chunk<T>::fma(w10, t10, aq);
            }
            Chunk<T>::fma(w11, t11, aq);
        }
    }
}

// The samples of one lane's ray inside one slab, staged as tap pairs (16-bit storage,
// four images per chunk): per sample the four bilinear weights are formed in the
// staging frame exactly as in slab_samples, rounded to the storage type in two pairs
// (row cy: taps cx, cx+1; row cy+1: the same columns), and each image takes one
// dot2 per row from one 16-byte read per plane and row.
template <typename T, int BC, int PITCH, int SH>
__device__ __forceinline__ void slab_samples_pair(const uint4 *lane_lds, int pitch, int plane_chunks,
                                                  double fxa, double fya, double sx, double sy,
                                                  int cnt, float *part) {
    constexpr int CH = Pair<T>::kImages;
    constexpr int PLANES = BC / CH;
    if (PITCH > 0) {
        pitch = PITCH;
        plane_chunks = (SH + 3) * PITCH;
    }
    const char *base = reinterpret_cast<const char *>(lane_lds);
    const unsigned row_bytes = (unsigned)pitch * 16u, plane_bytes = (unsigned)plane_chunks * 16u;
    const float end = (float)cnt, fxa32 = (float)fxa, fya32 = (float)fya;
    const float sx32 = (float)sx, sy32 = (float)sy;
    for (float jf = 0.0f; jf < end; jf += 1.0f) {
        const float px = fmaf(jf, sx32, fxa32), py = fmaf(jf, sy32, fya32);
        const int cx = (int)px, cy = (int)py;                       // px, py >= 1 - 1e-6
        const float fx = __builtin_amdgcn_fractf(px), fy = __builtin_amdgcn_fractf(py);
        const float gb = 1.0f - fy;
        const float w01 = __fmul_rn(fx, gb), w11 = __fmul_rn(fx, fy);
        const uint32_t wt = Pair<T>::weights(gb - w01, w01), wb = Pair<T>::weights(fy - w11, w11);
        const char *p0 = base + ((unsigned)__mul24(cy, pitch) + (unsigned)cx) * 16u;
#pragma unroll
        for (int q = 0; q < PLANES; ++q) {
            const uint4 t0 = *reinterpret_cast<const uint4 *>(p0 + q * plane_bytes);
            const uint4 t1 = *reinterpret_cast<const uint4 *>(p0 + q * plane_bytes + row_bytes);
            float *aq = part + q * CH;
            aq[0] = Pair<T>::dot2(t1.x, wb, Pair<T>::dot2(t0.x, wt, aq[0]));
            aq[1] = Pair<T>::dot2(t1.y, wb, Pair<T>::dot2(t0.y, wt, aq[1]));
            aq[2] = Pair<T>::dot2(t1.z, wb, Pair<T>::dot2(t0.z, wt, aq[2]));
            aq[3] = Pair<T>::dot2(t1.w, wb, Pair<T>::dot2(t0.w, wt, aq[3]));
        }
    }
}

// One block processes one work item (up to C::kWaves angles x 64 bins) x BC images,
// C = Source::Cfg the tiling.  The rays march through the image in slabs of
// C::kSlabH rows (or columns); per slab the block stages the slab's pixel window
// into LDS as 16-byte chunks holding Chunk<T>::kImages images each ("planes"),
// then every lane walks its ray's samples inside the slab.  A sample costs one
// address and weight computation shared by the BC images and four 16-byte LDS
// reads per plane.  The split of each ray's samples between slabs is fixed by
// FP64 boundary crossings (consistent across slabs); each lane's anchor cell in the
// slab is found in FP64 and its samples are FP32 offsets from it, so the weights'
// accuracy does not depend on where in the image the slab lies.
// PITCH > 0 (march-frame sources only): tile_t is that compile-time pitch.
template <typename T, int BC, class Source, int PITCH = 0>
__device__ __forceinline__ void fwd_item(const Geom &g, const FwdItem &it, const int2 *__restrict__ ranges,
                                         const ImageSet<T, BC> &imgs, const Source &src, int tile_t,
                                         uint4 *lds) {
    using C = typename Source::Cfg;
    constexpr int SH = C::kSlabH;
    static_assert(PITCH == 0 || Source::kMarchFrame, "a fixed pitch needs the march frame");
    if (PITCH > 0) tile_t = PITCH;
    const int plane_chunks = (SH + 3) * tile_t;

    // rays of the item -> lanes: each 16-lane quarter of a wave takes C::kQBins
    // neighbouring bins x C::kQAngles neighbouring angles, so the quarter's taps fall on
    // nearby columns (distinct LDS banks) and its rays have similar lengths; a wave is 4
    // quarters along the bins, 64 / (4 C::kQBins) waves cover the 64 bins
    constexpr int kWavesPerGroup = 16 / C::kQBins;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q16 = lane & 15;
    const int ai = C::kQAngles * (wave / kWavesPerGroup) + q16 / C::kQBins;
    const int di = 4 * C::kQBins * (wave % kWavesPerGroup) + C::kQBins * (lane >> 4) + q16 % C::kQBins;
    const bool active = ai < it.na && di < it.nd;
    const int a = it.a0 + min(ai, it.na - 1), d = it.d0 + min(di, it.nd - 1);
    const int n = g.n;

    // the lane's ray, oriented so that the march coordinate grows with the sample index
    double4 r = ray_params(g, a, d);
    const double sm_raw = it.axis ? r.z : r.w;
    if (sm_raw < 0.0) { r.z = -r.z; r.w = -r.w; }
    const double inv_sm = 1.0 / fabs(sm_raw);
    int jlo, jhi;
    support_range(r, n, jlo, jhi);
    // staging frame: the march frame swaps x and y for items marching along x
    const bool swap = Source::kMarchFrame && it.axis;
    if (swap) r = make_double4(r.y, r.x, r.w, r.z);
    const int faxis = Source::kMarchFrame ? 0 : it.axis;
    const double om = faxis ? r.x : r.y;
    const int pitch = faxis ? (SH + 3) : tile_t;

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int si = 0; si < it.nslab; ++si) {
        const int2 tr = ranges[it.range + si];
        if (tr.x > tr.y) continue;                      // uniform over the block
        const int m_lo = -1 + (it.slab0 + si) * SH;
        // tile element (0, 0) sits at frame pixel (ox0, oy0); tile is rows x cols pixels
        const int ox0 = faxis ? m_lo - 1 : tr.x;
        const int oy0 = faxis ? tr.x : m_lo - 1;
        const int cols = faxis ? SH + 3 : tr.y - tr.x + 1;
        const int rows = faxis ? tr.y - tr.x + 1 : SH + 3;

        __syncthreads();                                // previous slab fully consumed
        src.stage(lds, plane_chunks, pitch, ox0, oy0, rows, cols, it.axis);
        __syncthreads();

        // samples of this ray whose march coordinate lies in [m_lo, m_lo + SH)
        const int jb = max(jlo, (int)ceil(((double)m_lo - om) * inv_sm));
        const int je = min(jhi + 1, (int)ceil(((double)(m_lo + SH) - om) * inv_sm));
        if (jb >= je) continue;
        // anchor: one cell below the lowest cell over the slab's samples, so that every
        // sample offset is >= 1 in FP64 (>= 1 - 2e-6 once stepped in FP32, so
        // truncation is still floor) and small
        const double px64 = fma((double)jb, r.z, r.x) - (double)ox0;
        const double py64 = fma((double)jb, r.w, r.y) - (double)oy0;
        const double lx64 = fma((double)(je - 1 - jb), r.z, px64);
        const double ly64 = fma((double)(je - 1 - jb), r.w, py64);
        const double bx = floor(fmin(px64, lx64)) - 1.0, by = floor(fmin(py64, ly64)) - 1.0;
        const uint4 *lane_lds = lds + ((int)by * pitch + (int)bx);
        // the slab's samples are summed separately and then added to the ray total
        // (two-level summation keeps FP32 rounding of long rays small)
        float part[BC];
#pragma unroll
        for (int i = 0; i < BC; ++i) part[i] = 0.0f;
        if constexpr (Source::kPairs)
            slab_samples_pair<T, BC, PITCH, SH>(lane_lds, pitch, plane_chunks, px64 - bx, py64 - by,
                                            r.z, r.w, je - jb, part);
        else if (swap)
            slab_samples<T, BC, Source::kMarchFrame, PITCH, SH>(lane_lds, pitch, plane_chunks,
                                                            px64 - bx, py64 - by, r.z, r.w,
                                                            je - jb, part);
        else
            slab_samples<T, BC, false, PITCH, SH>(lane_lds, pitch, plane_chunks, px64 - bx, py64 - by,
                                              r.z, r.w, je - jb, part);
#pragma unroll
        for (int i = 0; i < BC; ++i) acc[i] += part[i];
    }
    if (!active) return;
#pragma unroll
    for (int i = 0; i < BC; ++i)
        if (i < imgs.count)
            Store<T>::store(imgs.out[i] + (size_t)a * g.det_count + d, acc[i] * imgs.scale[i]);
}

// ------------------------------------------------------------------ backprojection
// Sinogram staging sources.  For angles a0 .. a0+na-1 of a block, both fill the
// window of W bins starting at bin wlo_s[al] of angle a0+al (zero outside the
// detector) into LDS chunk planes: chunk (plane q, angle al, bin j) at
// q * per_plane + al * W + j.

// From the callers' sinograms (BC per-image pointers): one (angle, bin) pair per
// thread, one scalar load per image.
template <typename T, int BC>
struct SinoPointerSource {
    static constexpr bool kPairs = false;
    const T *const *img;
    int D;
    __device__ __forceinline__ void stage(uint4 *lds, int a0, int na, int W, const int *wlo_s,
                                          int per_plane) const {
        constexpr int CH = Chunk<T>::kImages;
        constexpr int PLANES = BC / CH;
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
                    const T val = img[q * CH + e][off];   // always a valid address
                    v[e] = inside ? val : Chunk<T>::zero();
                }
                lds[q * per_plane + al * W + j] = Chunk<T>::pack(v);
            }
        }
    }
};

// From the interleaved copy of the batch's sinograms, [groups][A][D + 2W] chunks of
// Chunk<T>::kImages images with W zero bins on either side: one 16-byte copy per
// chunk.  A window starting below -W or above D lies wholly in the zero region and is
// read from the nearest padded position instead.  Each thread owns up to kSlots
// fixed (plane, bin) slots of the window, set up once per block.  PAIRS (16-bit
// storage): the copy holds tap pairs, chunk j = bins j and j + 1 of four images.
template <typename T, int BC, bool PAIRS = false>
struct SinoInterleavedSource {
    static constexpr int kSlots = 4;
    static constexpr bool kPairs = PAIRS;
    const uint4 *base;     // first plane of the block's images
    int plane_stride;      // chunks between planes (A * (D + 2W))
    int D, Dp;             // detector bins, padded row length D + 2W
    int src_off[kSlots], lds_off[kSlots], slots;

    // slot k of this thread: element f = threadIdx + 256 k of the (plane, bin) window
    __device__ __forceinline__ void setup(int W, int per_plane) {
        constexpr int PLANES = BC / (PAIRS ? 4 : Chunk<T>::kImages);
        slots = 0;
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int f = (int)threadIdx.x + 256 * k;
            const int q = f / W, j = f - q * W;
            src_off[k] = q * plane_stride + W + j;
            lds_off[k] = q * per_plane + j;
            if (f < PLANES * W) slots = k + 1;
        }
    }
    __device__ __forceinline__ void stage(uint4 *lds, int a0, int na, int W, const int *wlo_s,
                                          int /*per_plane*/) const {
        for (int al = 0; al < na; ++al) {
            const int w0 = min(max(wlo_s[al], -W), D);
            const uint4 *row = base + (size_t)(a0 + al) * Dp + w0;
            uint4 *drow = lds + al * W;
#pragma unroll
            for (int k = 0; k < kSlots; ++k)
                if (k < slots) drow[lds_off[k]] = row[src_off[k]];
        }
    }
    // Asynchronous staging of the windows of na angles (lds_copy16_async: 16 bytes per
    // lane straight into LDS at a wave-uniform base + 16 * lane): angle-major layout
    // dst[al][plane][bin], angle stride PLANES * W, so element f = threadIdx + 256 k of
    // an angle is the lane's slot of a contiguous wave row.  Lanes past the window
    // (f >= PLANES * W) are masked off.
    __device__ __forceinline__ void issue(uint4 *dst, int a0, int na, int W, const int *wlo) const {
        constexpr int PLANES = BC / (PAIRS ? 4 : Chunk<T>::kImages);
        const int pw = PLANES * W;
        const int wave = (int)threadIdx.x & ~63;
        for (int al = 0; al < na; ++al) {
            const int w0 = min(max(wlo[al], -W), D);
            const uint4 *row = base + (size_t)(a0 + al) * Dp + w0;
#pragma unroll
            for (int k = 0; k < kSlots; ++k)
                if (k < slots) lds_copy16_async(row + src_off[k], dst + al * pw + 256 * k + wave);
        }
    }
    // Same with the planes P chunks apart (P >= W, a compile-time pitch): element
    // f = q * P + j (plane q, bin j < W) of angle al at dst[al * PLANES * P + f]; the
    // slots j >= W are left as they are (never read).
    template <int P>
    __device__ __forceinline__ void issue_pitched(uint4 *dst, int a0, int na, int W, const int *wlo) const {
        constexpr int PLANES = BC / (PAIRS ? 4 : Chunk<T>::kImages);
        constexpr int NS = (PLANES * P + 255) / 256;
        const int wave = (int)threadIdx.x & ~63;
        int off[NS];
        bool on[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int f = (int)threadIdx.x + 256 * k, q = f / P, j = f - q * P;
            on[k] = q < PLANES && j < W;
            off[k] = q * plane_stride + W + j;
        }
        for (int al = 0; al < na; ++al) {
            const int w0 = min(max(wlo[al], -W), D);
            const uint4 *row = base + (size_t)(a0 + al) * Dp + w0;
#pragma unroll
            for (int k = 0; k < NS; ++k)
                if (on[k]) lds_copy16_async(row + off[k], dst + al * PLANES * P + 256 * k + wave);
        }
    }
};

// NB candidate-bin weights of one (pixel, angle) applied to the tap-pair chunks of
// PLANES planes (four images each): chunk i of `row` holds bins lb + i and lb + i + 1,
// so the chunks at offsets 0, 2, 4, ... cover the candidates two at a time (a missing
// last partner gets weight 0) and each image takes one dot2 per chunk.  Planes run in
// a register pipeline as in the single-pixel chunks' loop.  PP: chunks between planes
// (0: `pp` at run time).
template <typename T, int PLANES, int NB, int PP>
__device__ __forceinline__ void bp_apply_pairs(const float *wgt, const uint4 *row, float *part,
                                               int pp = PP) {
    constexpr int NP = (NB + 1) / 2;
    if (PP > 0) pp = PP;
    uint32_t wp[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) wp[i] = Pair<T>::weights(wgt[2 * i], 2 * i + 1 < NB ? wgt[2 * i + 1] : 0.0f);
    uint4 cur[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) cur[i] = row[2 * i];
#pragma unroll
    for (int qq = 0; qq < PLANES; ++qq) {
        uint4 nxt[NP];
        if (qq + 1 < PLANES) {
#pragma unroll
            for (int i = 0; i < NP; ++i) nxt[i] = row[(qq + 1) * pp + 2 * i];
        }
        float *aq = part + qq * 4;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            aq[0] = Pair<T>::dot2(cur[i].x, wp[i], aq[0]);
            aq[1] = Pair<T>::dot2(cur[i].y, wp[i], aq[1]);
            aq[2] = Pair<T>::dot2(cur[i].z, wp[i], aq[2]);
            aq[3] = Pair<T>::dot2(cur[i].w, wp[i], aq[3]);
        }
        if (qq + 1 < PLANES) {
#pragma unroll
            for (int i = 0; i < NP; ++i) cur[i] = nxt[i];
        }
    }
}

// Parallel beam, one (pixel, angle): the NB x NK lattice samples (bin d, step k)
// whose bilinear footprint can cover the pixel.  The pixel's continuous lattice
// coordinates (u*, v*) are formed in FP64 from the angle's constants; candidates
// d = floor(u* - hu) + 1 + i, k = floor(v* - hv) + 1 + j; their offsets from the pixel
// are small FP32 numbers, so the tent weights are accurate to FP32 rounding.  Returns
// the first candidate bin, wgt[i] the summed weight of bin d + i.
template <int NB, int NK>
__device__ __forceinline__ int par_candidates(const Geom &g, const BpAngle &ba, double qx, double qy, float sp,
                                              float dt, float *wgt) {
    // continuous bin (u) and step (v) coordinates of the pixel centre
    const double u = fma(qx, ba.cu, fma(qy, ba.su, g.half_d));
    const double v = fma(qy, ba.cv, -qx * ba.sv);
    const double db = floor(u - ba.hu), kb = floor(v - ba.hv);
    // offset of candidate (d = db+1+i, k = kb+1+j) from the pixel, along u and v
    const float e0 = (float)(db + 1.0 - u) * sp, t0 = (float)(kb + 1.0 - v) * dt;
    float dx_i = fmaf(e0, ba.cf, -t0 * ba.sf), dy_i = fmaf(e0, ba.sf, t0 * ba.cf);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        float dx = dx_i, dy = dy_i, w = 0.0f;
#pragma unroll
        for (int jj = 0; jj < NK; ++jj) {
            const float tx = __builtin_amdgcn_fmed3f(1.0f - fabsf(dx), 0.0f, 1.0f);
            const float ty = __builtin_amdgcn_fmed3f(1.0f - fabsf(dy), 0.0f, 1.0f);
            w = fmaf(tx, ty, w);
            dx += ba.vx;
            dy += ba.vy;
        }
        wgt[i] = w;
        dx_i += ba.ux;
        dy_i += ba.uy;
    }
    return (int)db + 1;
}

// NB candidate-bin weights applied to the 16-byte chunks (Chunk<T>::kImages images
// each) of PLANES planes PP chunks apart, bins lb .. lb + NB - 1 at row[0 .. NB - 1]:
// planes in a register pipeline, the next plane's NB chunks read while the current
// plane's are applied, so LDS latency overlaps the multiply-adds.
template <typename T, int PLANES, int NB, int PP>
__device__ __forceinline__ void bp_apply_chunks(const float *wgt, const uint4 *row, float *part) {
    constexpr int CH = Chunk<T>::kImages;
    uint4 cur[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) cur[i] = row[i];
#pragma unroll
    for (int qq = 0; qq < PLANES; ++qq) {
        uint4 nxt[NB];
        if (qq + 1 < PLANES) {
#pragma unroll
            for (int i = 0; i < NB; ++i) nxt[i] = row[(qq + 1) * PP + i];
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) Chunk<T>::fma(wgt[i], cur[i], part + qq * CH);
        if (qq + 1 < PLANES) {
#pragma unroll
            for (int i = 0; i < NB; ++i) cur[i] = nxt[i];
        }
    }
}

// Parallel beam.  One block = a 16x16 pixel tile (lane <-> pixel) x BC images.
// Angles are processed in blocks of AB: for each, the block stages into LDS
// the window of W bins its tile can touch, as 16-byte chunks of Chunk<T>::kImages
// images ("planes").  Each pixel then finds, per angle, the lattice samples whose
// bilinear footprint covers it (par_candidates) and applies the NB bin weights to BC
// images with 16-byte LDS reads.  No atomics.  This form stages each block between
// barriers (the caller's sinograms, and the uneven batches).
template <typename T, int BC, int NB, int NK, int AB, class Source>
__device__ __forceinline__ void bp_tile_par(const Geom &g, int tile, const ImageSet<T, BC> &imgs,
                                            const Source &src, int W, uint4 *lds) {
    __shared__ int wlo_s[AB];
    constexpr int CH = Source::kPairs ? 4 : Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    static_assert(BC % CH == 0, "BC must be a multiple of the images per chunk");
    const int n = g.n, A = g.n_angles;
    const int tiles_x = (n + kBpTile - 1) / kBpTile;
    const int tx0 = (tile % tiles_x) * kBpTile, ty0 = (tile / tiles_x) * kBpTile;
    const int c = tx0 + (threadIdx.x % kBpTile), r = ty0 + (threadIdx.x / kBpTile);
    const double qx = (double)c - g.cn, qy = (double)r - g.cn;
    const double tcx = tx0 + 0.5 * (kBpTile - 1) - g.cn, tcy = ty0 + 0.5 * (kBpTile - 1) - g.cn;
    // planes at a fixed pitch (W <= kBpWinPar): the reads below use immediate offsets
    constexpr int per_plane = AB * kBpWinPar;
    const float dt = (float)g.step, sp = (float)g.spacing;

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int a0 = 0; a0 < A; a0 += AB) {
        const int na = min(AB, A - a0);
        __syncthreads();                                // previous block consumed
        if (threadIdx.x < na) {
            const BpAngle ba = g.bpa[a0 + threadIdx.x];
            const double uc = fma(tcx, ba.cu, fma(tcy, ba.su, g.half_d));
            wlo_s[threadIdx.x] = (int)floor(uc - (0.5 * (kBpTile - 1) + 1.0) * ba.hu) - 1;
        }
        __syncthreads();
        src.stage(lds, a0, na, W, wlo_s, per_plane);
        __syncthreads();

        // the angle block's contributions are summed separately, then added to the
        // pixel total (two-level summation keeps FP32 rounding small); with 64 images
        // per lane the partial sums would halve the occupancy, so they go straight to
        // the totals
        constexpr bool kTwoLevel = BC <= 32;
        float part_buf[kTwoLevel ? BC : 1];
        float *part = kTwoLevel ? part_buf : acc;
        if (kTwoLevel) {
#pragma unroll
            for (int i = 0; i < BC; ++i) part[i] = 0.0f;
        }
        for (int al = 0; al < na; ++al) {
            float wgt[NB];
            int lb = par_candidates<NB, NK>(g, g.bpa[a0 + al], qx, qy, sp, dt, wgt) - wlo_s[al];
            lb = min(max(lb, 0), W - NB);               // memory safety; real pixels are inside
            const uint4 *row = lds + al * W + lb;
            if constexpr (Source::kPairs)
                bp_apply_pairs<T, PLANES, NB, per_plane>(wgt, row, part);
            else
                bp_apply_chunks<T, PLANES, NB, per_plane>(wgt, row, part);
        }
        if (kTwoLevel) {
#pragma unroll
            for (int i = 0; i < BC; ++i) acc[i] += part[i];
        }
    }
    if (c >= n || r >= n) return;
#pragma unroll
    for (int i = 0; i < BC; ++i)
        if (i < imgs.count)
            Store<T>::store(imgs.out[i] + (size_t)r * n + c, acc[i] * imgs.scale[i]);
}

// Parallel beam from the interleaved copy, with the sinogram windows double-buffered
// as in bp_tile_fan_async: the next block's copies (lds_copy16_async) run while this
// block is applied.  Windows at a fixed plane pitch of kBpWinPar chunks, angle stride
// PLANES * kBpWinPar (both immediates in the reads).  The blocks' angle constants are
// copied into LDS the same way two blocks ahead (triple-buffered), so the steps before
// each barrier touch no global memory: after the wait for this wave's copies, the first
// AB threads form the next block's window bounds from LDS.  Same arithmetic and
// summation order as bp_tile_par.
template <typename T, int BC, int NB, int NK, int AB, bool PAIRS>
__device__ __forceinline__ void bp_tile_par_async(const Geom &g, int tile, const ImageSet<T, BC> &imgs,
                                                  const SinoInterleavedSource<T, BC, PAIRS> &src, int W,
                                                  uint4 *lds) {
    __shared__ int wlo_s[3][AB];
    __shared__ BpAngle bpa_s[3][AB];
    constexpr int CH = PAIRS ? 4 : Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    static_assert(BC % CH == 0, "BC must be a multiple of the images per chunk");
    static_assert(AB * sizeof(BpAngle) / 16 <= 64, "one wave copies a block's angle constants");
    constexpr int AS = PLANES * kBpWinPar;             // chunks per staged angle
    const int n = g.n, A = g.n_angles;
    const int tiles_x = (n + kBpTile - 1) / kBpTile;
    const int tx0 = (tile % tiles_x) * kBpTile, ty0 = (tile / tiles_x) * kBpTile;
    const int c = tx0 + (threadIdx.x % kBpTile), r = ty0 + (threadIdx.x / kBpTile);
    const double qx = (double)c - g.cn, qy = (double)r - g.cn;
    const double tcx = tx0 + 0.5 * (kBpTile - 1) - g.cn, tcy = ty0 + 0.5 * (kBpTile - 1) - g.cn;
    const float dt = (float)g.step, sp = (float)g.spacing;
    // copies of the constants of the angle block starting at a (na angles) into slot
    // k, by the lanes of wave 0
    auto copy_angles = [&](int a, int na, int k) {
        constexpr int kChunks = sizeof(BpAngle) / 16;
        if (threadIdx.x < 64 && (int)threadIdx.x < na * kChunks)
            lds_copy16_async(reinterpret_cast<const uint4 *>(g.bpa + a) + threadIdx.x,
                             reinterpret_cast<uint4 *>(&bpa_s[k][0]));
    };
    // first bin of the tile's window at angle al of slot k (thread al < AB)
    auto bounds = [&](int k, int al) {
        const BpAngle &ba = bpa_s[k][al];
        const double uc = fma(tcx, ba.cu, fma(tcy, ba.su, g.half_d));
        wlo_s[k][al] = (int)floor(uc - (0.5 * (kBpTile - 1) + 1.0) * ba.hu) - 1;
    };

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    const int nblk = (A + AB - 1) / AB;
    copy_angles(0, min(AB, A), 0);
    if (A > AB) copy_angles(AB, min(AB, A - AB), 1);
    __builtin_amdgcn_s_waitcnt(0);
    if ((int)threadIdx.x < min(AB, A)) bounds(0, threadIdx.x);
    __syncthreads();
    src.template issue_pitched<kBpWinPar>(lds, 0, min(AB, A), W, wlo_s[0]);
    for (int b = 0; b < nblk; ++b) {
        const int a0 = b * AB, na = min(AB, A - a0), nn = min(AB, A - a0 - AB), n2 = min(AB, A - a0 - 2 * AB);
        const int cur = b & 1, tb = b % 3, tn = (b + 1) % 3;
        const uint4 *sino_cur = lds + cur * AB * AS;
        uint4 *sino_next = lds + (cur ^ 1) * AB * AS;
        __builtin_amdgcn_s_waitcnt(0);                 // this wave's copies have landed: block
                                                       // b's windows, block b + 1's constants
        if ((int)threadIdx.x < nn) bounds(tn, threadIdx.x);
        __syncthreads();                               // ... and everyone's; next bounds written
        // the next block's windows and the constants two blocks ahead are copied while
        // this block is applied
        if (nn > 0) src.template issue_pitched<kBpWinPar>(sino_next, a0 + AB, nn, W, wlo_s[tn]);
        if (n2 > 0) copy_angles(a0 + 2 * AB, n2, (b + 2) % 3);

        constexpr bool kTwoLevel = BC <= 32;
        float part_buf[kTwoLevel ? BC : 1];
        float *part = kTwoLevel ? part_buf : acc;
        if (kTwoLevel) {
#pragma unroll
            for (int i = 0; i < BC; ++i) part[i] = 0.0f;
        }
        for (int al = 0; al < na; ++al) {
            float wgt[NB];
            int lb = par_candidates<NB, NK>(g, bpa_s[tb][al], qx, qy, sp, dt, wgt) - wlo_s[tb][al];
            lb = min(max(lb, 0), W - NB);               // memory safety; real pixels are inside
            const uint4 *row = sino_cur + al * AS + lb;
            if constexpr (PAIRS)
                bp_apply_pairs<T, PLANES, NB, kBpWinPar>(wgt, row, part);
            else
                bp_apply_chunks<T, PLANES, NB, kBpWinPar>(wgt, row, part);
        }
        if (kTwoLevel) {
#pragma unroll
            for (int i = 0; i < BC; ++i) acc[i] += part[i];
        }
    }
    if (c >= n || r >= n) return;
#pragma unroll
    for (int i = 0; i < BC; ++i)
        if (i < imgs.count)
            Store<T>::store(imgs.out[i] + (size_t)r * n + c, acc[i] * imgs.scale[i]);
}

// The angles al of one staged block with NBX candidate bins per pixel (NBX <= the
// plan's bin count: the caller checked that NBX bins cover every footprint of the tile
// at these angles).  FP32 throughout: the first candidate bin comes from the projection
// of the pixel centre and its first-order half-width with a margin (0.05 bins + 1%)
// far above FP32 rounding (~1e-4 bins); each bin's ray is a lattice point near the
// tile and its step, in tile coordinates (|values| <= ~50 px), so the offsets of the
// candidate samples from the pixel carry ~1e-6 pixel of rounding, as in the parallel
// kernel.
template <typename T, int BC, int NBX, int NK, bool PAIRS>
__device__ __forceinline__ void fan_angle_block(const Geom &g, const double2 *trig, int na, int W, const int *wlo_s,
                                                const float4 *rays_s, const uint4 *lds, int per_plane,
                                                int as, float qx, float qy, float lx, float ly, float is2,
                                                float *part, int skip = 0) {
    constexpr int CH = PAIRS ? 4 : Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    const float sd = (float)g.sd, k_sde = (float)(g.sde * g.inv_spacing), hd = (float)g.half_d;
    for (int al = 0; al < na; ++al) {
        const double2 cs64 = trig[al];
        const float cx = (float)cs64.x, sy = (float)cs64.y;
        // detector coordinate of the pixel centre and its gradient (bins per pixel)
        const float pu = fmaf(qx, cx, qy * sy), pv = fmaf(-qx, sy, qy * cx);
        const float near = sd + pv;
        // hardware reciprocal (1 ulp): den only places the candidate bins, whose
        // margin is ~1e5 times larger than its error
        const float den = __builtin_amdgcn_rcpf(near);
        const float sb = fmaf(k_sde * pu, den, hd);
        const float k2 = k_sde * den * den;
        const float gsx = k2 * fmaf(cx, near, pu * sy), gsy = k2 * fmaf(sy, near, -pu * cx);
        const float hb = fabsf(gsx) + fabsf(gsy);
        const int dfirst = (int)ceilf(sb - hb * 1.01f - 0.05f) + skip;
        int lb = dfirst - wlo_s[al];
        lb = min(max(lb, 0), W - NBX);              // memory safety; real pixels are inside
        float wgt[NBX];
#pragma unroll
        for (int i = 0; i < NBX; ++i) {
            const float4 rp = rays_s[al * W + lb + i];
            const float ex = rp.x - lx, ey = rp.y - ly;                  // lattice point - pixel
            const float kc = -fmaf(ex, rp.z, ey * rp.w) * is2;           // pixel along the ray
            const float hk = (fabsf(rp.z) + fabsf(rp.w)) * is2;
            const float k1 = floorf(kc - hk) + 1.0f;
            float dx = fmaf(k1, rp.z, ex), dy = fmaf(k1, rp.w, ey);
            float w = 0.0f;
#pragma unroll
            for (int jj = 0; jj < NK; ++jj) {
                const float tx = __builtin_amdgcn_fmed3f(1.0f - fabsf(dx), 0.0f, 1.0f);
                const float ty = __builtin_amdgcn_fmed3f(1.0f - fabsf(dy), 0.0f, 1.0f);
                w = fmaf(tx, ty, w);
                dx += rp.z;
                dy += rp.w;
            }
            wgt[i] = w;
        }
        const uint4 *row = lds + al * as + lb;
        if constexpr (PAIRS) {
            bp_apply_pairs<T, PLANES, NBX, 0>(wgt, row, part, per_plane);
        } else {
            // planes in a register pipeline (the next plane's NBX chunks are read while
            // the current plane's are applied): with few waves per SIMD the LDS latency
            // is otherwise exposed once per plane
            uint4 cur[NBX];
#pragma unroll
            for (int i = 0; i < NBX; ++i) cur[i] = row[i];
#pragma unroll
            for (int qq = 0; qq < PLANES; ++qq) {
                uint4 nxt[NBX];
                if (qq + 1 < PLANES) {
#pragma unroll
                    for (int i = 0; i < NBX; ++i) nxt[i] = row[(qq + 1) * per_plane + i];
                }
#pragma unroll
                for (int i = 0; i < NBX; ++i) Chunk<T>::fma(wgt[i], cur[i], part + qq * CH);
                if (qq + 1 < PLANES) {
#pragma unroll
                    for (int i = 0; i < NBX; ++i) cur[i] = nxt[i];
                }
            }
        }
    }
}

// Bin window start of a 16x16 tile at an angle of cos/sin cs (the projections of the corners of its
// footprint) and the candidate bins a footprint can need there:
// |grad s| <= SE/(S+v) sqrt(1 + (u/(S+v))^2) with v the smallest and |u| the largest
// over the corners (both linear).  FP64, one thread per angle.
template <int NB>
__device__ __forceinline__ void fan_tile_bounds(const Geom &g, int tx0, int ty0, double2 cs, int *wlo, int *nb) {
    double lo = 1e30, vmin = 1e30, umax = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double px = tx0 - 1.0 + ((k & 1) ? kBpTile + 1.0 : 0.0) - g.cn;
        const double py = ty0 - 1.0 + ((k & 2) ? kBpTile + 1.0 : 0.0) - g.cn;
        const double pu = fma(px, cs.x, py * cs.y), pv = fma(-px, cs.y, py * cs.x);
        lo = fmin(lo, g.sde * pu / (g.sd + pv) * g.inv_spacing + g.half_d);
        vmin = fmin(vmin, pv);
        umax = fmax(umax, fabs(pu));
    }
    *wlo = (int)floor(lo) - 1;
    const double near = g.sd + vmin, ratio = umax / near;
    const double grad = g.sde / near * sqrt(1.0 + ratio * ratio);
    const double span = 2.0 * 1.4142135623730951 * grad * g.inv_spacing * 1.01 + 0.1;
    *nb = near > 0.0 ? (int)floor(span) + 1 : NB;
}

// The rays of the bin windows of na angles into rays_s[al * W + j]: each ray's samples
// are o + k s (index coordinates, FP64); staged is its lattice point nearest the tile
// centre, relative to the tile origin, and its step, in FP32.  A bin outside the
// detector gets a ray far from every pixel (weight 0).
__device__ __forceinline__ float4 fan_tile_ray(const Geom &g, const double4 &rp, int tx0, int ty0) {
    const double tcx = tx0 + 0.5 * (kBpTile - 1), tcy = ty0 + 0.5 * (kBpTile - 1);
    const double k0 = rint(fma(tcx - rp.x, rp.z, (tcy - rp.y) * rp.w) * g.inv_step * g.inv_step);
    return make_float4((float)(fma(k0, rp.z, rp.x) - tx0), (float)(fma(k0, rp.w, rp.y) - ty0), (float)rp.z,
                       (float)rp.w);
}
__device__ __forceinline__ void fan_stage_rays(const Geom &g, int a0, int na, int W, const int *wlo_s,
                                               int tx0, int ty0, float4 *rays_s) {
    const int D = g.det_count;
    for (int p = threadIdx.x; p < na * W; p += 256) {
        const int al = p / W, j = p - al * W;
        const int d = wlo_s[al] + j;
        float4 v = make_float4(-1e9f, -1e9f, 0.0f, 0.0f);
        if ((unsigned)d < (unsigned)D) v = fan_tile_ray(g, g.rays[(size_t)(a0 + al) * D + d], tx0, ty0);
        rays_s[al * W + j] = v;
    }
}

// Fan beam.  Same tiling as the parallel kernel; every bin has its own ray, so the
// block also stages the rays of its bin window (each as its lattice point nearest the
// tile, relative to the tile, and its step, in FP32).  Per (pixel, angle) the
// candidate bins are those within the projected half-width of the pixel's footprint
// around the projection of its centre (first-order bound plus a margin far larger
// than the footprint's curvature); per bin, the NK candidate samples around the
// pixel's position along that ray are evaluated from small FP32 offsets, as in the
// parallel kernel.  The plan's NB bins cover the worst magnification in the image;
// per block of angles the tile's own bound (its footprint's smallest distance to the
// source and largest lateral offset) usually needs only 4 (96% of the blocks of a
// 512^2 image at S = 1000, E = 500, 1.5-pixel bins), and only the other blocks run a
// second pass over the next 2.  This form stages each block of AB angles between
// barriers (the caller's sinograms, and the uneven batches).
template <typename T, int BC, int NB, int NK, int AB, class Source>
__device__ __forceinline__ void bp_tile_fan(const Geom &g, int tile, const ImageSet<T, BC> &imgs,
                                            const Source &src, int W, uint4 *lds) {
    __shared__ int wlo_s[AB];
    __shared__ int nb_s[AB];
    constexpr int CH = Source::kPairs ? 4 : Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    static_assert(BC % CH == 0, "BC must be a multiple of the images per chunk");
    const int n = g.n, A = g.n_angles;
    const int tiles_x = (n + kBpTile - 1) / kBpTile;
    const int tx0 = (tile % tiles_x) * kBpTile, ty0 = (tile / tiles_x) * kBpTile;
    const int c = tx0 + (threadIdx.x % kBpTile), r = ty0 + (threadIdx.x / kBpTile);
    const float qx = (float)((double)c - g.cn), qy = (float)((double)r - g.cn);
    const float lx = (float)(c - tx0), ly = (float)(r - ty0);
    const int per_plane = AB * W;
    float4 *rays_s = reinterpret_cast<float4 *>(lds + PLANES * per_plane);
    const float is2 = (float)(g.inv_step * g.inv_step);

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    for (int a0 = 0; a0 < A; a0 += AB) {
        const int na = min(AB, A - a0);
        __syncthreads();
        if (threadIdx.x < na)
            fan_tile_bounds<NB>(g, tx0, ty0, g.trig[a0 + threadIdx.x], &wlo_s[threadIdx.x], &nb_s[threadIdx.x]);
        __syncthreads();
        src.stage(lds, a0, na, W, wlo_s, per_plane);
        fan_stage_rays(g, a0, na, W, wlo_s, tx0, ty0, rays_s);
        int nb_block = 0;
        for (int al = 0; al < na; ++al) nb_block = max(nb_block, nb_s[al]);
        __syncthreads();

        // two-level summation as in the parallel kernel (single level at 64 images)
        constexpr bool kTwoLevel = BC <= 32;
        float part_buf[kTwoLevel ? BC : 1];
        float *part = kTwoLevel ? part_buf : acc;
        if (kTwoLevel) {
#pragma unroll
            for (int i = 0; i < BC; ++i) part[i] = 0.0f;
        }
        // candidate bins: four, and for the angle blocks whose bound needs more, two
        // more in a second pass (one 4-bin body keeps the registers of the wide lanes
        // at three waves per SIMD, where a 6-bin body needed two)
        fan_angle_block<T, BC, 4, NK, Source::kPairs>(g, g.trig + a0, na, W, wlo_s, rays_s, lds, per_plane, W, qx,
                                                      qy, lx, ly, is2, part);
        if (NB > 4 && nb_block > 4)
            fan_angle_block<T, BC, 2, NK, Source::kPairs>(g, g.trig + a0, na, W, wlo_s, rays_s, lds, per_plane, W, qx,
                                                          qy, lx, ly, is2, part, 4);
        if (kTwoLevel) {
#pragma unroll
            for (int i = 0; i < BC; ++i) acc[i] += part[i];
        }
    }
    if (c >= n || r >= n) return;
#pragma unroll
    for (int i = 0; i < BC; ++i)
        if (i < imgs.count)
            Store<T>::store(imgs.out[i] + (size_t)r * n + c, acc[i] * imgs.scale[i]);
}

// Fan beam from the interleaved copy, with the sinogram windows double-buffered: the
// copy of the next block of AB angles goes straight from global memory into the other
// LDS buffer (asynchronous, see SinoInterleavedSource::issue) while this block is
// applied, so the block stalls on staging only when the copy outlasts the arithmetic.
// The block's cos/sin pairs are copied the same way two blocks ahead and its raw FP64
// rays (32 bytes per bin) one block ahead, so the steps before each barrier touch no
// global memory: after the wait for its own copies each wave turns the raw rays it
// copied into tile-relative FP32 rays (a wave copies whole rays), and the first AB
// threads bound the next block's windows from the cos/sin in LDS.  Same arithmetic,
// candidate bins and summation order as bp_tile_fan.  Buffers: sinogram windows and
// FP32 rays 2 each (angle-major windows, angle stride PLANES * W), raw rays 1 (consumed
// before the barrier after which it is refilled), window bounds and cos/sin 3 (a
// block's are overwritten two iterations after they are written, when no wave can
// still apply that block).
template <typename T, int BC, int NB, int NK, int AB, bool PAIRS>
__device__ __forceinline__ void bp_tile_fan_async(const Geom &g, int tile, const ImageSet<T, BC> &imgs,
                                                  const SinoInterleavedSource<T, BC, PAIRS> &src, int W,
                                                  uint4 *lds) {
    __shared__ int wlo_s[3][AB];
    __shared__ int nb_s[3][AB];
    __shared__ double2 trig_s[3][AB];
    constexpr int CH = PAIRS ? 4 : Chunk<T>::kImages;
    constexpr int PLANES = BC / CH;
    static_assert(BC % CH == 0, "BC must be a multiple of the images per chunk");
    const int n = g.n, A = g.n_angles, D = g.det_count;
    const int tiles_x = (n + kBpTile - 1) / kBpTile;
    const int tx0 = (tile % tiles_x) * kBpTile, ty0 = (tile / tiles_x) * kBpTile;
    const int c = tx0 + (threadIdx.x % kBpTile), r = ty0 + (threadIdx.x / kBpTile);
    const float qx = (float)((double)c - g.cn), qy = (float)((double)r - g.cn);
    const float lx = (float)(c - tx0), ly = (float)(r - ty0);
    const float is2 = (float)(g.inv_step * g.inv_step);
    const int pw = PLANES * W;                         // chunks per staged angle
    // LDS: sinogram windows 2 x AB * pw chunks, FP32 rays 2 x AB * W, raw rays AB * W x 32 B
    float4 *rays0 = reinterpret_cast<float4 *>(lds + 2 * AB * pw);
    uint4 *raw = lds + 2 * AB * pw + 2 * AB * W;
    // cos/sin of the block starting at a (na angles) into slot k, by the lanes of wave 0
    auto copy_trig = [&](int a, int na, int k) {
        if ((int)threadIdx.x < na)
            lds_copy16_async(reinterpret_cast<const uint4 *>(g.trig + a) + threadIdx.x,
                             reinterpret_cast<uint4 *>(&trig_s[k][0]));
    };
    // raw rays of the block's windows: bin p = al * W + j is chunks 2p and 2p + 1 of
    // `raw`; chunk e = threadIdx + 256 i is lane e mod 64 of a contiguous wave row, so
    // each wave copies whole rays (bins outside the detector are not copied)
    auto copy_rays = [&](int a, int na, const int *wlo) {
        for (int e = threadIdx.x; e < 2 * na * W; e += 256) {
            const int p = e >> 1, al = p / W, d = wlo[al] + (p - al * W);
            if ((unsigned)d < (unsigned)D)
                lds_copy16_async(reinterpret_cast<const uint4 *>(g.rays + (size_t)(a + al) * D + d) + (e & 1),
                                 raw + (e - (threadIdx.x & 63)));
        }
    };
    // the raw rays this thread's wave copied, as tile-relative FP32 rays
    auto finish_rays = [&](int na, const int *wlo, float4 *rays_s) {
        for (int e = threadIdx.x; e < 2 * na * W; e += 256) {
            if (e & 1) continue;
            const int p = e >> 1, al = p / W, d = wlo[al] + (p - al * W);
            float4 v = make_float4(-1e9f, -1e9f, 0.0f, 0.0f);
            if ((unsigned)d < (unsigned)D) v = fan_tile_ray(g, reinterpret_cast<const double4 *>(raw)[p], tx0, ty0);
            rays_s[p] = v;
        }
    };

    float acc[BC];
#pragma unroll
    for (int i = 0; i < BC; ++i) acc[i] = 0.0f;

    const int nblk = (A + AB - 1) / AB;
    copy_trig(0, min(AB, A), 0);
    if (A > AB) copy_trig(AB, min(AB, A - AB), 1);
    __builtin_amdgcn_s_waitcnt(0);
    if ((int)threadIdx.x < min(AB, A))
        fan_tile_bounds<NB>(g, tx0, ty0, trig_s[0][threadIdx.x], &wlo_s[0][threadIdx.x], &nb_s[0][threadIdx.x]);
    __syncthreads();
    src.issue(lds, 0, min(AB, A), W, wlo_s[0]);
    copy_rays(0, min(AB, A), wlo_s[0]);
    for (int b = 0; b < nblk; ++b) {
        const int a0 = b * AB, na = min(AB, A - a0), nn = min(AB, A - a0 - AB), n2 = min(AB, A - a0 - 2 * AB);
        const int cur = b & 1, tb = b % 3, tn = (b + 1) % 3;
        const uint4 *sino_cur = lds + cur * AB * pw;
        uint4 *sino_next = lds + (cur ^ 1) * AB * pw;
        float4 *rays_cur = rays0 + cur * AB * W;
        __builtin_amdgcn_s_waitcnt(0);                 // this wave's copies have landed: block
                                                       // b's windows and raw rays, b + 1's cos/sin
        finish_rays(na, wlo_s[tb], rays_cur);
        if ((int)threadIdx.x < nn)
            fan_tile_bounds<NB>(g, tx0, ty0, trig_s[tn][threadIdx.x], &wlo_s[tn][threadIdx.x],
                                &nb_s[tn][threadIdx.x]);
        __syncthreads();                               // ... and everyone's; rays and bounds written
        int nb_block = 0;
        for (int al = 0; al < na; ++al) nb_block = max(nb_block, nb_s[tb][al]);
        // the next block's windows and raw rays, and the cos/sin two blocks ahead, are
        // copied while this block is applied
        if (nn > 0) {
            src.issue(sino_next, a0 + AB, nn, W, wlo_s[tn]);
            copy_rays(a0 + AB, nn, wlo_s[tn]);
        }
        if (n2 > 0) copy_trig(a0 + 2 * AB, n2, (b + 2) % 3);

        constexpr bool kTwoLevel = BC <= 32;
        float part_buf[kTwoLevel ? BC : 1];
        float *part = kTwoLevel ? part_buf : acc;
        if (kTwoLevel) {
#pragma unroll
            for (int i = 0; i < BC; ++i) part[i] = 0.0f;
        }
        fan_angle_block<T, BC, 4, NK, PAIRS>(g, trig_s[tb], na, W, wlo_s[tb], rays_cur, sino_cur, W, pw, qx, qy,
                                             lx, ly, is2, part);
        if (NB > 4 && nb_block > 4)
            fan_angle_block<T, BC, 2, NK, PAIRS>(g, trig_s[tb], na, W, wlo_s[tb], rays_cur, sino_cur, W, pw, qx,
                                                 qy, lx, ly, is2, part, 4);
        if (kTwoLevel) {
#pragma unroll
            for (int i = 0; i < BC; ++i) acc[i] += part[i];
        }
    }
    if (c >= n || r >= n) return;
#pragma unroll
    for (int i = 0; i < BC; ++i)
        if (i < imgs.count)
            Store<T>::store(imgs.out[i] + (size_t)r * n + c, acc[i] * imgs.scale[i]);
}

}  // namespace radon
