// Uneven-batch descriptors shared by the host planner and the persistent kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "radon_common.hpp"
#include "radon_launch.hpp"

namespace radon {

constexpr int kBatchFwdImages = 8;    // images per lane in the batched forward units
constexpr int kBatchBpImages = 32;    // images per lane in the batched backprojection units

// One job of an uneven batch as the device sees it.
struct BatchJob {
    Geom g;
    const FwdItem *items;     // forward plan items
    const int2 *ranges;       // forward plan slab ranges
    int tile_t;               // forward LDS tile extent
    int window;               // backprojection bin window
    int bins;                 // backprojection candidate bins (fan)
    int batch;                // images in the job
    const void *in;
    void *out;
    float scale_dt;           // scale * step
};

// One unit of work: forward (job, plan item, first image); backprojection
// (job, pixel tile, first image).
struct WorkUnit {
    int job, unit, b0, pad;
};

struct BatchLaunch {
    const BatchJob *jobs = nullptr;   // device
    const WorkUnit *work = nullptr;   // device
    int *counter = nullptr;           // device work counter
    int n_work = 0;
    int grid = 0;
    size_t lds = 0;
};

// direction 0 = forward, 1 = backprojection.  Launches the counter reset and the
// persistent kernel on stream s (no allocation, no synchronisation).
hipError_t launch_batched(int direction, int dtype, const BatchLaunch &L, hipStream_t s);

// Resident blocks per CU of the persistent kernel for a dynamic LDS size.
int batched_blocks_per_cu(int direction, int dtype, size_t lds);

}  // namespace radon
