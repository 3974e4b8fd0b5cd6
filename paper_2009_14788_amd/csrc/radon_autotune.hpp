// Autotuned launch shapes per (plan, storage type, batch size class).
#pragma once

#include "radon_launch.hpp"
#include "radon_plan.hpp"

namespace radon {

// Batch size class: the next power of two (shapes are tuned per class).
int batch_class(int batch);

// Time the candidate shapes of both directions for `plan` at this storage type and
// batch (or read them from the RADON_TUNE_CACHE file).  Synchronises the device and
// allocates temporary buffers.  Returns 0 on success.
int autotune(Plan &plan, int dtype, int batch, void *ws, size_t ws_bytes, TunedShapes &out);

}  // namespace radon
