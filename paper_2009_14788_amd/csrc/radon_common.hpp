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
// expression from the same FP32 ray parameters, and the bilinear weights as the
// products (1-fx or fx) * (1-fy or fy) of the same factors, so the two kernels
// use bit-identical matrix entries and differ only in summation order.
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
    int n;              // image side N
    int n_angles;       // A
    int det_count;      // D
    int fan;            // 0 parallel, 1 fan
    float cn;           // (N-1)/2
    float half_d;       // (D-1)/2
    float spacing;      // detector spacing
    float inv_spacing;
    float step;         // sample spacing along a ray
    float inv_step;
    float sd;           // fan: source distance S
    float sde;          // fan: S + E
    const float2 *trig; // [A] (cos, sin) of each angle, FP32 rounded from FP64
    const float4 *rays; // fan: [A*D] (ox, oy, sx, sy), FP32 rounded from FP64
};

// Ray parameters of (angle a, bin d).
__device__ __forceinline__ float4 ray_params(const Geom &g, int a, int d) {
    if (g.fan) return g.rays[(size_t)a * g.det_count + d];
    float2 cs = g.trig[a];
    float s = ((float)d - g.half_d) * g.spacing;
    return make_float4(fmaf(s, cs.x, g.cn), fmaf(s, cs.y, g.cn), -cs.y * g.step, cs.x * g.step);
}

// Integer k range [klo, khi] (a superset) of the samples with px, py in (-1, N),
// i.e. inside the support of the bilinear interpolant.  Empty when klo > khi.
__device__ __forceinline__ void sample_range(const float4 &r, int n, int &klo, int &khi) {
    float lo = -3.0e7f, hi = 3.0e7f;
    const float fn = (float)n;
    // x axis
    if (fabsf(r.z) > 1e-12f) {
        float inv = 1.0f / r.z;
        float t1 = (-1.0f - r.x) * inv, t2 = (fn - r.x) * inv;
        lo = fmaxf(lo, fminf(t1, t2));
        hi = fminf(hi, fmaxf(t1, t2));
    } else if (!(r.x > -1.0f && r.x < fn)) {
        lo = 1.0f; hi = -1.0f;
    }
    if (fabsf(r.w) > 1e-12f) {
        float inv = 1.0f / r.w;
        float t1 = (-1.0f - r.y) * inv, t2 = (fn - r.y) * inv;
        lo = fmaxf(lo, fminf(t1, t2));
        hi = fminf(hi, fmaxf(t1, t2));
    } else if (!(r.y > -1.0f && r.y < fn)) {
        lo = 1.0f; hi = -1.0f;
    }
    if (lo > hi) { klo = 1; khi = 0; return; }
    klo = (int)floorf(lo);
    khi = (int)ceilf(hi);
}

// Tent factor for the pixel at integer index q of a sample at fractional index p:
// max(0, 1 - |p - q|); equals 1-frac(p) for q = floor(p) and frac(p) for q = floor(p)+1.
__device__ __forceinline__ float tent(float p, float q) {
    return fmaxf(0.0f, 1.0f - fabsf(p - q));
}

}  // namespace radon
