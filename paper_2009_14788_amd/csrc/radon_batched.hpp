// Uneven-batch descriptors shared by the host planner and the persistent kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "radon_common.hpp"
#include "radon_launch.hpp"

namespace radon {

constexpr int kBatchBpNarrow = 8;      // images per lane in small backprojection units
constexpr int kBatchBpMid = 16;        // images per lane in medium backprojection units
constexpr int kBatchBpWide = 32;       // images per lane in large backprojection units

// One geometry of an uneven batch as the device sees it (shared by every job of
// the batch that uses that geometry).
struct BatchJob {
    Geom g;
    const FwdItem *items;     // forward plan items
    const int2 *ranges;       // forward plan slab ranges
    int tile_t;               // forward LDS tile extent
    int window;               // backprojection bin window
    int bins;                 // backprojection candidate bins (fan)
    int pad;
};

// Up to kBatchBpWide images of one geometry, possibly from different jobs: input
// and output base pointers and the output scale (scale * step) of each.  Entries
// past `count` repeat the last valid input.
struct ImageGroup {
    const void *in[kBatchBpWide];
    void *out[kBatchBpWide];
    float scale[kBatchBpWide];
    int count;
    int pad[3];
};

// One unit of work: forward (geometry, plan item, image group); backprojection
// (geometry, pixel tile, image group).  `wide` (backprojection): 0 = kBatchBpNarrow,
// 1 = kBatchBpWide, 2 = kBatchBpMid images per lane; 0 for the forward.
struct WorkUnit {
    int job, unit, group, wide;
};

struct BatchLaunch {
    const BatchJob *jobs = nullptr;     // device
    const ImageGroup *groups = nullptr; // device
    const WorkUnit *work = nullptr;     // device
    int *counter = nullptr;             // device work counter
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
