// Shared device-side definitions of the Radon kernels (gfx950).
//
// Coordinates.  Kernels work in "index coordinates": a point (px, py) lies at
// fractional column px and fractional row py, so pixel (r, c) has its centre at
// (c, r).  The centred coordinates of the operator (pixel centre at
// (c-(N-1)/2, r-(N-1)/2)) are shifted by cN = (N-1)/2.
//
// A ray is (ox, oy) = its foot point F in index coordinates and (sx, sy) =
// step * its unit direction w; sample k sits at (ox + k sx, oy + k sy).  The kernels
// form these positions independently and to different roundings: the direct kernels
// in FP64 per sample; the tiled forward finds each lane's first sample in a slab in
// FP64 and steps the following ones as FP32 offsets from it (below ~2e-6 pixel of
// error); the tiled backprojection forms each pixel's coordinates along and across
// the rays of an angle in FP64 and the tent arguments as small FP32 differences.
// Forward and backprojection are therefore transposes of each other up to FP32
// rounding of the weights (the dot-product gap is at that level, not zero).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace radon {

enum Dtype { F32 = 0, F16 = 1, BF16 = 2 };

struct bf16_t { uint16_t bits; };

// ---------------------------------------------------------------- storage types
template <typename T> struct Store;

template <> struct Store<float> {
    static __device__ __forceinline__ float load(const float *p) { return *p; }
    static __device__ __forceinline__ void store(float *p, float v) { *p = v; }
};

template <> struct Store<__half> {
    static __device__ __forceinline__ float load(const __half *p) { return __half2float(*p); }
    static __device__ __forceinline__ void store(__half *p, float v) { *p = __float2half_rn(v); }
};

template <> struct Store<bf16_t> {
    static __device__ __forceinline__ float load(const bf16_t *p) {
        return __uint_as_float(((uint32_t)p->bits) << 16);
    }
    // round to nearest even; NaN stays NaN
    static __device__ __forceinline__ void store(bf16_t *p, float v) {
        uint32_t u = __float_as_uint(v);
        uint16_t out;
        if ((u & 0x7fffffffu) > 0x7f800000u) {
            out = (uint16_t)((u >> 16) | 0x40u);
        } else {
            u += 0x7fffu + ((u >> 16) & 1u);
            out = (uint16_t)(u >> 16);
        }
        p->bits = out;
    }
};

// ---------------------------------------------------------------- 16-byte LDS chunks
// A chunk holds one pixel of kImages images (4 FP32 or 8 FP16/BF16 values); the
// tiled kernels move image and sinogram data through LDS in such chunks so that
// every LDS read is a full 16-byte lane access.
template <typename T> struct Chunk;

template <> struct Chunk<float> {
    static constexpr int kImages = 4;
    static __device__ __forceinline__ float zero() { return 0.0f; }
    static __device__ __forceinline__ uint4 pack(const float *v) {
        return make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                          __float_as_uint(v[3]));
    }
    static __device__ __forceinline__ void fma(float w, const uint4 &t, float *acc) {
        acc[0] = fmaf(w, __uint_as_float(t.x), acc[0]);
        acc[1] = fmaf(w, __uint_as_float(t.y), acc[1]);
        acc[2] = fmaf(w, __uint_as_float(t.z), acc[2]);
        acc[3] = fmaf(w, __uint_as_float(t.w), acc[3]);
    }
};

__device__ __forceinline__ float half_lo(uint32_t u) {
    return __half2float(__ushort_as_half((unsigned short)(u & 0xffffu)));
}
__device__ __forceinline__ float half_hi(uint32_t u) {
    return __half2float(__ushort_as_half((unsigned short)(u >> 16)));
}

template <> struct Chunk<__half> {
    static constexpr int kImages = 8;
    static __device__ __forceinline__ __half zero() { return __ushort_as_half(0); }
    static __device__ __forceinline__ uint4 pack(const __half *v) {
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            w[k] = (uint32_t)__half_as_ushort(v[2 * k]) | ((uint32_t)__half_as_ushort(v[2 * k + 1]) << 16);
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
    static __device__ __forceinline__ void fma(float w, const uint4 &t, float *acc) {
        const uint32_t u[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc[2 * k] = fmaf(w, half_lo(u[k]), acc[2 * k]);
            acc[2 * k + 1] = fmaf(w, half_hi(u[k]), acc[2 * k + 1]);
        }
    }
};

template <> struct Chunk<bf16_t> {
    static constexpr int kImages = 8;
    static __device__ __forceinline__ bf16_t zero() { return bf16_t{0}; }
    static __device__ __forceinline__ uint4 pack(const bf16_t *v) {
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = (uint32_t)v[2 * k].bits | ((uint32_t)v[2 * k + 1].bits << 16);
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
    static __device__ __forceinline__ void fma(float w, const uint4 &t, float *acc) {
        const uint32_t u[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc[2 * k] = fmaf(w, __uint_as_float(u[k] << 16), acc[2 * k]);
            acc[2 * k + 1] = fmaf(w, __uint_as_float(u[k] & 0xffff0000u), acc[2 * k + 1]);
        }
    }
};

// ---------------------------------------------------------------- tap-pair chunks
// 16-bit storage in "tap pairs": a 16-byte chunk holds two horizontally adjacent
// pixels (x, x+1) of four images, one 32-bit word per image (pixel x in the low
// half).  One dot2 instruction (v_dot2c_f32_f16 / v_dot2c_f32_bf16: both 16-bit
// products are exact in FP32 and added to the FP32 accumulator) then applies the two
// bilinear weights of a row of taps, so a bilinear sample costs two instructions per
// image instead of four multiply-adds.  The weights are rounded to the storage type
// (round to nearest even) for that.  Along a ray whose direction is close to an axis
// the fractional sample positions change slowly, so these rounding errors are
// correlated from sample to sample and do not average out: the sum carries up to the
// weights' relative rounding (2^-12 in FP16, 2^-9 in BF16), the same order as the
// rounding of the stored output.
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

template <typename T> struct Pair;

template <> struct Pair<__half> {
    static constexpr int kImages = 4;
    // (lo, hi) rounded to FP16 and packed, lo in bits 0..15
    static __device__ __forceinline__ uint32_t weights(float lo, float hi) {
        const f16x2_t v = {(_Float16)lo, (_Float16)hi};
        return __builtin_bit_cast(uint32_t, v);
    }
    static __device__ __forceinline__ float dot2(uint32_t taps, uint32_t w, float acc) {
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, taps), __builtin_bit_cast(f16x2_t, w),
                                      acc, false);
    }
    static __device__ __forceinline__ uint32_t bits(__half h) { return __half_as_ushort(h); }
};

template <> struct Pair<bf16_t> {
    static constexpr int kImages = 4;
    static __device__ __forceinline__ uint32_t weights(float lo, float hi) {
        const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
        return __builtin_bit_cast(uint32_t, v);
    }
    static __device__ __forceinline__ float dot2(uint32_t taps, uint32_t w, float acc) {
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, taps),
                                               __builtin_bit_cast(bf16x2_t, w), acc, false);
    }
    static __device__ __forceinline__ uint32_t bits(bf16_t h) { return h.bits; }
};

// ---------------------------------------------------------------- geometry
struct Geom {
    int n;               // image side N
    int n_angles;        // A
    int det_count;       // D
    int fan;             // 0 parallel, 1 fan
    double cn;           // (N-1)/2
    double half_d;       // (D-1)/2
    double spacing;      // detector spacing
    double inv_spacing;
    double step;         // sample spacing along a ray
    double inv_step;
    double sd;           // fan: source distance S
    double sde;          // fan: S + E
    const double2 *trig; // [A] (cos, sin) of each angle
    const double4 *rays; // fan: [A*D] (ox, oy, sx, sy)
    const struct BpAngle *bpa;  // parallel: [A] per-angle backprojection constants
};

// Per-angle constants of the parallel-beam backprojection, formed on the host in FP64
// once per geometry: the pixel at centred coordinates (qx, qy) has bin coordinate
// u = qx*cu + qy*su + (D-1)/2 and step coordinate v = qy*cv - qx*sv.
// 80 bytes (five 16-byte chunks), so the double-buffered kernels copy a block's
// constants into LDS with 16-byte asynchronous copies.
struct alignas(16) BpAngle {
    double cu, su;   // cos / spacing, sin / spacing
    double cv, sv;   // cos / step, sin / step
    double hu, hv;   // (|cos| + |sin|) / spacing, (|cos| + |sin|) / step
    float cf, sf;    // cos, sin
    float ux, uy;    // one bin along the detector: spacing * (cos, sin)
    float vx, vy;    // one step along the ray: step * (-sin, cos)
};
static_assert(sizeof(BpAngle) == 80, "five 16-byte chunks per angle");

// Ray parameters of (angle a, bin d), FP64: foot point in index coordinates and
// step * unit direction.  Sample positions are formed in FP64 and only their
// fractional parts (the bilinear weights) drop to FP32, so a sample's weights are
// accurate to FP32 rounding wherever it lies in the image.
__device__ __forceinline__ double4 ray_params(const Geom &g, int a, int d) {
    if (g.fan) return g.rays[(size_t)a * g.det_count + d];
    const double2 cs = g.trig[a];
    const double s = ((double)d - g.half_d) * g.spacing;
    return make_double4(fma(s, cs.x, g.cn), fma(s, cs.y, g.cn), -cs.y * g.step, cs.x * g.step);
}

// Integer k range [klo, khi] (a superset) of the samples with px, py in (-1, N),
// i.e. inside the support of the bilinear interpolant.  Empty when klo > khi.
__device__ __forceinline__ void sample_range(const double4 &r, int n, int &klo, int &khi) {
    double lo = -1.0e9, hi = 1.0e9;
    const double fn = (double)n;
    const double o[2] = {r.x, r.y}, w[2] = {r.z, r.w};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (fabs(w[i]) > 1e-300) {
            const double inv = 1.0 / w[i];
            const double t1 = (-1.0 - o[i]) * inv, t2 = (fn - o[i]) * inv;
            lo = fmax(lo, fmin(t1, t2));
            hi = fmin(hi, fmax(t1, t2));
        } else if (!(o[i] > -1.0 && o[i] < fn)) {
            lo = 1.0;
            hi = -1.0;
        }
    }
    if (lo > hi) { klo = 1; khi = 0; return; }
    klo = (int)floor(lo);
    khi = (int)ceil(hi);
}

// Exact k range [klo, khi] of the samples strictly inside the support box
// (-1, N)^2 (up to FP64 rounding at the boundary, where a sample's weight is ~0).
__device__ __forceinline__ void support_range(const double4 &r, int n, int &klo, int &khi) {
    double lo = -1.0e9, hi = 1.0e9;
    const double fn = (double)n;
    const double o[2] = {r.x, r.y}, w[2] = {r.z, r.w};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (fabs(w[i]) > 1e-300) {
            const double inv = 1.0 / w[i];
            const double t1 = (-1.0 - o[i]) * inv, t2 = (fn - o[i]) * inv;
            lo = fmax(lo, fmin(t1, t2));
            hi = fmin(hi, fmax(t1, t2));
        } else if (!(o[i] > -1.0 && o[i] < fn)) {
            lo = 1.0;
            hi = -1.0;
        }
    }
    if (lo > hi) { klo = 1; khi = 0; return; }
    klo = (int)ceil(lo);
    khi = (int)floor(hi);
}

// Sample position along one axis: integer cell index (floor) and FP32 fraction.
// The pixel at index floor(p) gets weight 1 - frac, the next one frac.
struct Cell {
    int i;
    float f;
};
__device__ __forceinline__ Cell cell_of(double p) {
    const double fl = floor(p);
    Cell c;
    c.i = (int)fl;
    c.f = (float)(p - fl);
    return c;
}

// Weight that a sample in cell c gives pixel index q along one axis.
__device__ __forceinline__ float axis_weight(const Cell &c, int q) {
    return q == c.i ? 1.0f - c.f : (q == c.i + 1 ? c.f : 0.0f);
}

}  // namespace radon
