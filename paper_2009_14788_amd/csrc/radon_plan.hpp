// Per-geometry plan: device tables and the launch shapes chosen for them.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <utility>
#include <vector>

#include "../../include/radon.h"
#include "radon_common.hpp"
#include "radon_launch.hpp"

namespace radon {

struct PlanKey {
    int device = 0;
    int beam = 0;
    int n = 0;
    int det_count = 0;
    double det_spacing = 0, source_distance = 0, det_distance = 0, step = 0;
    std::vector<double> angles;
    bool operator==(const PlanKey &o) const;
};

struct PlanKeyHash {
    size_t operator()(const PlanKey &k) const;
};

// Launch shapes chosen by the autotuner for one (storage type, batch class).
struct TunedShapes {
    bool valid = false;
    int fwd_variant = VARIANT_TILED, bp_variant = VARIANT_TILED;
    int fwd_images = 8, fwd_stage = 1, fwd_tiling = 0;
    int bp_images = 32, bp_angles = 8, bp_stage = 1;
};

struct Plan {
    int device = 0;
    Geom geom{};
    double2 *trig = nullptr;  // device [A]
    double4 *rays = nullptr;  // device [A*D], fan beam only
    BpAngle *bpa = nullptr;   // device [A], parallel beam only
    // tiled forward work per tiling (kFwdTiling[t]); n_items = 0 where it does not apply
    FwdItem *fwd_items[kFwdTilings] = {};  // device, tiled forward work items
    int2 *fwd_ranges[kFwdTilings] = {};    // device, per item and slab transverse ranges
    FwdWork fwd_work[kFwdTilings];
    std::vector<FwdItem> fwd_items_host;   // host copy of tiling 0 (work-unit costs of uneven batches)
    BpWork bp_work;
    bool no_interleave = false;            // stage the forward from the caller's images
    LaunchShape fwd_shape, bp_shape;       // defaults
    size_t key_hash = 0;
    std::map<std::pair<int, int>, TunedShapes> tuned;   // (dtype, batch class) -> shapes
    Plan() = default;
    Plan(const Plan &) = delete;
    Plan &operator=(const Plan &) = delete;
    ~Plan();
};

int validate(const radon_geometry_t *g);
PlanKey make_key(const radon_geometry_t *g, int device);
int get_plan(const radon_geometry_t *g, hipStream_t stream, Plan **out);

// Library-owned workspace of one (device, stream), grown to `need` bytes outside stream
// capture (a buffer it replaces stays allocated until radon_release_plans); *have
// receives its size, which may be smaller than need under capture.  NULL on failure.
void *stream_workspace(hipStream_t stream, size_t need, size_t *have);
// Frees the shearlet plans (called by radon_release_plans after a device sync).
void release_shearlet_plans();

}  // namespace radon
