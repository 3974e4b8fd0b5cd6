// Shared device-side definitions of the Radon kernels (gfx950).
//
// Coordinates.  Kernels work in "index coordinates": a point (px, py) lies at
// fractional column px and fractional row py, so pixel (r, c) has its centre at
// (c, r).  The centred coordinates of the operator (pixel centre at
// (c-(N-1)/2, r-(N-1)/2)) are shifted by cN = (N-1)/2.
//
// A ray is (ox, oy) = its foot point F in index coordinates and (sx, sy) =
// step * its unit direction w; sample k sits at (fma(k, sx, ox), fma(k, sy, oy)).
// Forward and backprojection evaluate sample positions with exactly this
// expression from the same ray parameters, and the bilinear weights as the
// products (1-fx or fx) * (1-fy or fy) of the same FP32 factors, so the two
// kernels use bit-identical sample weights and differ only in summation order.
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
};

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
