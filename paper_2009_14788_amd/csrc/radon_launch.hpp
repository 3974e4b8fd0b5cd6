// Host-side launch interface between the C ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "radon_common.hpp"

namespace radon {

// Launch shape of one direction, chosen per plan (fixed default or autotuned).
struct LaunchShape {
    int variant = 0;      // kernel family (0 = direct)
    int images = 4;       // images per thread
    int angles = 1;       // angles per block
    int rays = 256;       // rays (forward) or pixels (backprojection) per block
};

hipError_t launch_forward(const Geom &g, int dtype, const LaunchShape &shape, const void *x,
                          void *y, int batch, float scale, hipStream_t s);
hipError_t launch_backproject(const Geom &g, int dtype, const LaunchShape &shape,
                              const void *y, void *x, int batch, float scale, hipStream_t s);
hipError_t launch_dot_f64(const void *a, const void *b, long long n, int dtype, double *out,
                          double *partials, int n_partials, hipStream_t s);

}  // namespace radon
