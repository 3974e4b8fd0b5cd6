// C ABI of libradon.so: validation, per-geometry plans, dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <deque>
#include <map>
#include <memory>
#include <tuple>
#include <string>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/radon.h"
#include "radon_autotune.hpp"
#include "radon_batched.hpp"
#include "radon_filter.hpp"
#include "radon_launch.hpp"
#include "radon_plan.hpp"
#include "radon_shearlet.hpp"

namespace radon {

// ---------------------------------------------------------------- validation
int validate(const radon_geometry_t *g) {
    if (!g) return RADON_ERR_INVALID_ARG;
    if (g->beam != RADON_PARALLEL && g->beam != RADON_FANBEAM) return RADON_ERR_INVALID_ARG;
    if (g->image_size < 1 || g->n_angles < 1 || g->det_count < 1) return RADON_ERR_INVALID_ARG;
    // sizes whose index arithmetic would leave 32-bit float/int exactness
    if (g->image_size > 16384 || g->det_count > (1 << 20) || g->n_angles > (1 << 20) ||
        (int64_t)g->n_angles * g->det_count > INT32_MAX)
        return RADON_ERR_UNSUPPORTED;
    if (!g->angles) return RADON_ERR_INVALID_ARG;
    for (int a = 0; a < g->n_angles; ++a)
        if (!std::isfinite(g->angles[a])) return RADON_ERR_INVALID_ARG;
    if (!(g->det_spacing > 0.0) || !std::isfinite(g->det_spacing)) return RADON_ERR_INVALID_ARG;
    if (!(g->step > 0.0) || !std::isfinite(g->step)) return RADON_ERR_INVALID_ARG;
    // keep per-ray sample counts and sample indices well inside 32-bit range
    if (g->step < 1e-3 || g->step > 1e3 || g->det_spacing > 1e6) return RADON_ERR_UNSUPPORTED;
    if (g->beam == RADON_FANBEAM) {
        const double support = 0.5 * (g->image_size + 1) * std::sqrt(2.0);
        if (!(g->source_distance > support) || !std::isfinite(g->source_distance))
            return RADON_ERR_INVALID_ARG;
        if (!(g->det_distance >= 0.0) || !std::isfinite(g->det_distance))
            return RADON_ERR_INVALID_ARG;
    }
    return RADON_OK;
}

static int check_ptr(const void *p) {
    if (!p) return RADON_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(p) & 15u) return RADON_ERR_ALIGN;
    return RADON_OK;
}

static int check_dtype(int32_t dtype) {
    return (dtype == RADON_F32 || dtype == RADON_F16 || dtype == RADON_BF16) ? RADON_OK
                                                                             : RADON_ERR_INVALID_ARG;
}

// ---------------------------------------------------------------- plan cache
PlanKey make_key(const radon_geometry_t *g, int device) {
    PlanKey k;
    k.device = device;
    k.beam = g->beam;
    k.n = g->image_size;
    k.det_count = g->det_count;
    k.det_spacing = g->det_spacing;
    k.source_distance = g->beam == RADON_FANBEAM ? g->source_distance : 0.0;
    k.det_distance = g->beam == RADON_FANBEAM ? g->det_distance : 0.0;
    k.step = g->step;
    k.angles.assign(g->angles, g->angles + g->n_angles);
    return k;
}

size_t PlanKeyHash::operator()(const PlanKey &k) const {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    };
    mix(&k.device, sizeof k.device);
    mix(&k.beam, sizeof k.beam);
    mix(&k.n, sizeof k.n);
    mix(&k.det_count, sizeof k.det_count);
    mix(&k.det_spacing, sizeof k.det_spacing);
    mix(&k.source_distance, sizeof k.source_distance);
    mix(&k.det_distance, sizeof k.det_distance);
    mix(&k.step, sizeof k.step);
    mix(k.angles.data(), k.angles.size() * sizeof(double));
    return (size_t)h;
}

bool PlanKey::operator==(const PlanKey &o) const {
    return device == o.device && beam == o.beam && n == o.n && det_count == o.det_count &&
           det_spacing == o.det_spacing && source_distance == o.source_distance &&
           det_distance == o.det_distance && step == o.step && angles == o.angles;
}

Plan::~Plan() {
    if (trig) (void)hipFree(trig);
    if (rays) (void)hipFree(rays);
    if (bpa) (void)hipFree(bpa);
    for (int t = 0; t < kFwdTilings; ++t) {
        if (fwd_items[t]) (void)hipFree(fwd_items[t]);
        if (fwd_ranges[t]) (void)hipFree(fwd_ranges[t]);
    }
}

static std::mutex g_mutex;
static std::unordered_map<PlanKey, std::unique_ptr<Plan>, PlanKeyHash> g_plans;

// Scratch of the FP64 inner products, one set per (device, stream): calls on
// different streams may run at the same time, so they never share partial sums.
// The single-system partials are slots of pooled blocks, so a stream seen for the
// first time while it captures (a graph's own capture stream) takes a free slot
// without allocating; the per-system partials of radon_dot_f64_batched are grown
// outside capture only.  A replaced buffer stays allocated (a captured graph may
// still use it) until radon_release_plans.
constexpr int kDotPartials = 1024;   // doubles per single-system slot
constexpr int kDotSlots = 64;        // slots per pooled block
struct StreamScratch {
    double *dot_partials = nullptr;   // one slot of a DeviceScratch block
    double *row_partials = nullptr;   // per-system partials of radon_dot_f64_batched
    size_t row_count = 0;
};
struct DeviceScratch {
    std::vector<double *> dot_blocks; // kDotSlots slots of kDotPartials doubles each
    size_t dot_used = 0;
    std::vector<void *> retired;      // replaced per-system buffers
};
static std::unordered_map<int, DeviceScratch> g_scratch;
static std::map<std::pair<int, hipStream_t>, StreamScratch> g_stream_scratch;

static bool is_capturing(hipStream_t stream, int *rc) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    *rc = hipStreamIsCapturing(stream, &cap) == hipSuccess ? RADON_OK : RADON_ERR_HIP;
    return cap != hipStreamCaptureStatusNone;
}

// Host FP64 angle and ray tables.
// rays[a*D+d] = (ox, oy, sx, sy): foot point in index coordinates, step * direction.
static void fill_tables(const radon_geometry_t *g, std::vector<double2> &trig,
                        std::vector<double4> &rays) {
    const int A = g->n_angles, D = g->det_count;
    const double cn = 0.5 * (g->image_size - 1);
    trig.resize(A);
    for (int a = 0; a < A; ++a)
        trig[a] = make_double2(std::cos(g->angles[a]), std::sin(g->angles[a]));
    rays.resize((size_t)A * D);
    if (g->beam != RADON_FANBEAM) {
        for (int a = 0; a < A; ++a)
            for (int d = 0; d < D; ++d) {
                const double s = (d - 0.5 * (D - 1)) * g->det_spacing;
                const double c = trig[a].x, sn = trig[a].y;
                rays[(size_t)a * D + d] =
                    make_double4(std::fma(s, c, cn), std::fma(s, sn, cn), -sn * g->step, c * g->step);
            }
        return;
    }
    const double S = g->source_distance, E = g->det_distance;
    for (int a = 0; a < A; ++a) {
        const double ux = std::cos(g->angles[a]), uy = std::sin(g->angles[a]);
        const double vx = -uy, vy = ux;
        for (int d = 0; d < D; ++d) {
            const double s = (d - 0.5 * (D - 1)) * g->det_spacing;
            const double sx = -S * vx, sy = -S * vy;              // source
            const double ex = E * vx + s * ux, ey = E * vy + s * uy; // bin centre
            double wx = ex - sx, wy = ey - sy;
            const double len = std::sqrt(wx * wx + wy * wy);
            wx /= len;
            wy /= len;
            const double along = sx * wx + sy * wy;
            const double fx = sx - along * wx, fy = sy - along * wy; // foot point
            rays[(size_t)a * D + d] = make_double4(fx + cn, fy + cn, g->step * wx, g->step * wy);
        }
    }
}

static int build_plan(const radon_geometry_t *g, int device, std::unique_ptr<Plan> &out) {
    std::unique_ptr<Plan> p(new (std::nothrow) Plan());
    if (!p) return RADON_ERR_ALLOC;
    std::vector<double2> trig;
    std::vector<double4> rays;
    fill_tables(g, trig, rays);
    if (hipMalloc(&p->trig, trig.size() * sizeof(double2)) != hipSuccess) return RADON_ERR_ALLOC;
    if (hipMemcpy(p->trig, trig.data(), trig.size() * sizeof(double2), hipMemcpyHostToDevice) !=
        hipSuccess)
        return RADON_ERR_HIP;
    if (g->beam != RADON_FANBEAM) {
        // per-angle constants of the parallel backprojection
        std::vector<BpAngle> bpa(g->n_angles);
        for (int a = 0; a < g->n_angles; ++a) {
            const double c = trig[a].x, sn = trig[a].y, h = std::fabs(c) + std::fabs(sn);
            BpAngle &b = bpa[a];
            b.cu = c / g->det_spacing;
            b.su = sn / g->det_spacing;
            b.cv = c / g->step;
            b.sv = sn / g->step;
            b.hu = h / g->det_spacing;
            b.hv = h / g->step;
            b.cf = (float)c;
            b.sf = (float)sn;
            b.ux = (float)(g->det_spacing * c);
            b.uy = (float)(g->det_spacing * sn);
            b.vx = (float)(-g->step * sn);
            b.vy = (float)(g->step * c);
        }
        if (hipMalloc(&p->bpa, bpa.size() * sizeof(BpAngle)) != hipSuccess) return RADON_ERR_ALLOC;
        if (hipMemcpy(p->bpa, bpa.data(), bpa.size() * sizeof(BpAngle), hipMemcpyHostToDevice) !=
            hipSuccess)
            return RADON_ERR_HIP;
    }
    if (g->beam == RADON_FANBEAM) {
        if (hipMalloc(&p->rays, rays.size() * sizeof(double4)) != hipSuccess) return RADON_ERR_ALLOC;
        if (hipMemcpy(p->rays, rays.data(), rays.size() * sizeof(double4),
                      hipMemcpyHostToDevice) != hipSuccess)
            return RADON_ERR_HIP;
    }
    // tiled forward work items
    std::vector<FwdItem> items;
    std::vector<int2> ranges;
    int tile_t = 0;
    const char *force = std::getenv("RADON_VARIANT");
    const bool want_direct = force && std::strcmp(force, "direct") == 0;
    // tiled forward: one plan per tiling (tiling 0 decides whether the tiled kernels
    // apply at all; another tiling that does not fit keeps n_items = 0)
    for (int t = 0; t < kFwdTilings && !want_direct; ++t) {
        if (!plan_forward_tiles(g->image_size, g->n_angles, g->det_count, rays, kFwdTiling[t].slab_h,
                                kFwdTiling[t].waves, items, ranges, tile_t) ||
            items.empty()) {
            if (t == 0) break;
            continue;
        }
        // longest items first (slabs the item's rays cross): blocks are dispatched in
        // index order, so the short items fill the tail of the launch
        std::vector<int> slabs(items.size(), 0);
        for (size_t i = 0; i < items.size(); ++i)
            for (int si = 0; si < items[i].nslab; ++si)
                slabs[i] += ranges[items[i].range + si].x <= ranges[items[i].range + si].y;
        std::vector<size_t> order(items.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return slabs[a] > slabs[b]; });
        std::vector<FwdItem> sorted(items.size());
        for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];
        items.swap(sorted);
        if (hipMalloc(&p->fwd_items[t], items.size() * sizeof(FwdItem)) != hipSuccess)
            return RADON_ERR_ALLOC;
        if (hipMemcpy(p->fwd_items[t], items.data(), items.size() * sizeof(FwdItem),
                      hipMemcpyHostToDevice) != hipSuccess)
            return RADON_ERR_HIP;
        const size_t nr = std::max<size_t>(ranges.size(), 1);
        if (hipMalloc(&p->fwd_ranges[t], nr * sizeof(int2)) != hipSuccess) return RADON_ERR_ALLOC;
        if (!ranges.empty() && hipMemcpy(p->fwd_ranges[t], ranges.data(), ranges.size() * sizeof(int2),
                                         hipMemcpyHostToDevice) != hipSuccess)
            return RADON_ERR_HIP;
        FwdWork &w = p->fwd_work[t];
        w.items = p->fwd_items[t];
        w.ranges = p->fwd_ranges[t];
        w.n_items = (int)items.size();
        // LDS row pitch: 8 more than a multiple of 16 chunks, so the taps of lanes
        // whose samples sit in neighbouring rows land half a bank cycle apart
        w.tile_t = (tile_t + 15 - kFwdPitchMod) / 16 * 16 + kFwdPitchMod;
        if (t > 0) continue;
        p->fwd_items_host = items;
        p->fwd_shape.variant = VARIANT_TILED;
        const char *il = std::getenv("RADON_FWD_INTERLEAVE");
        p->no_interleave = il && std::strcmp(il, "0") == 0;
        const char *imgs = std::getenv("RADON_FWD_IMAGES");
        p->fwd_shape.images = (imgs && std::atoi(imgs) >= 16) ? 16 : 8;
        p->fwd_shape.angles = kFwdWaves;
        p->fwd_shape.rays = kFwdLanes;
        p->fwd_shape.tiling = 0;
    }
    // tiled backprojection
    if (!want_direct) {
        p->bp_work = plan_backproject(g->beam, g->image_size, trig, g->det_spacing, g->step,
                                      g->source_distance, g->det_distance);
        if (p->bp_work.window > 0) {
            p->bp_shape.variant = VARIANT_TILED;
            p->bp_shape.images = 32;
            p->bp_shape.angles = g->beam == RADON_FANBEAM ? kBpAnglesFan : kBpAngles;
            p->bp_shape.rays = kBpTile * kBpTile;
        }
    }
    Geom &G = p->geom;
    G.n = g->image_size;
    G.n_angles = g->n_angles;
    G.det_count = g->det_count;
    G.fan = g->beam == RADON_FANBEAM ? 1 : 0;
    G.cn = 0.5 * (g->image_size - 1);
    G.half_d = 0.5 * (g->det_count - 1);
    G.spacing = g->det_spacing;
    G.inv_spacing = 1.0 / g->det_spacing;
    G.step = g->step;
    G.inv_step = 1.0 / g->step;
    G.sd = g->source_distance;
    G.sde = g->source_distance + g->det_distance;
    G.trig = p->trig;
    G.rays = p->rays;
    G.bpa = p->bpa;
    p->device = device;
    out = std::move(p);
    return RADON_OK;
}

// Find the plan of g on the current device; build it unless the stream captures.
int get_plan(const radon_geometry_t *g, hipStream_t stream, Plan **out) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return RADON_ERR_NO_DEVICE;
    PlanKey key = make_key(g, device);
    std::lock_guard<std::mutex> lock(g_mutex);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.get();
        return RADON_OK;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return RADON_ERR_HIP;
    if (cap != hipStreamCaptureStatusNone) return RADON_ERR_NOT_PREPARED;
    std::unique_ptr<Plan> p;
    int rc = build_plan(g, device, p);
    if (rc != RADON_OK) return rc;
    p->key_hash = PlanKeyHash()(key);
    *out = p.get();
    g_plans.emplace(std::move(key), std::move(p));
    return RADON_OK;
}

// Workspace for the interleaved copy of a call's input batch (images for the
// forward, sinograms for the backprojection), one per (device, stream) so calls on
// different streams never share it; calls on one stream use it in stream order.  Grown on demand outside
// stream capture; a smaller buffer it replaces stays allocated (a captured graph may
// still use it) until radon_release_plans.  Under capture without a large enough
// workspace the forward stages straight from the caller's images instead.
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    std::vector<void *> retired;
};
static std::unordered_map<std::string, Workspace> g_workspaces;

void *stream_workspace(hipStream_t stream, size_t need, size_t *have) {
    *have = 0;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return nullptr;
    std::string key(reinterpret_cast<const char *>(&device), sizeof device);
    key.append(reinterpret_cast<const char *>(&stream), sizeof stream);
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace &w = g_workspaces[key];
    if (w.bytes < need) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
            return w.ptr ? (*have = w.bytes, w.ptr) : nullptr;
        void *p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) return w.ptr ? (*have = w.bytes, w.ptr) : nullptr;
        if (w.ptr) w.retired.push_back(w.ptr);
        w.ptr = p;
        w.bytes = need;
    }
    *have = w.bytes;
    return w.ptr;
}

static int dot_scratch(hipStream_t stream, double **out) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return RADON_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_mutex);
    StreamScratch &ss = g_stream_scratch[{device, stream}];
    if (!ss.dot_partials) {
        DeviceScratch &d = g_scratch[device];
        if (d.dot_used == d.dot_blocks.size() * kDotSlots) {
            int rc;
            const bool cap = is_capturing(stream, &rc);
            if (rc != RADON_OK) return rc;
            if (cap) return RADON_ERR_NOT_PREPARED;
            double *b = nullptr;
            if (hipMalloc(&b, (size_t)kDotSlots * kDotPartials * sizeof(double)) != hipSuccess)
                return RADON_ERR_ALLOC;
            d.dot_blocks.push_back(b);
        }
        ss.dot_partials = d.dot_blocks[d.dot_used / kDotSlots] + (d.dot_used % kDotSlots) * kDotPartials;
        ++d.dot_used;
    }
    *out = ss.dot_partials;
    return RADON_OK;
}

static int row_scratch(hipStream_t stream, size_t count, double **out) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return RADON_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_mutex);
    StreamScratch &ss = g_stream_scratch[{device, stream}];
    if (ss.row_count < count) {
        int rc;
        const bool cap = is_capturing(stream, &rc);
        if (rc != RADON_OK) return rc;
        if (cap) return RADON_ERR_NOT_PREPARED;
        double *p = nullptr;
        if (hipMalloc(&p, count * sizeof(double)) != hipSuccess) return RADON_ERR_ALLOC;
        if (ss.row_partials) g_scratch[device].retired.push_back(ss.row_partials);
        ss.row_partials = p;
        ss.row_count = count;
    }
    *out = ss.row_partials;
    return RADON_OK;
}

// ---------------------------------------------------------------- FBP filter tables
// Frequency response and twiddles of one (device, padded length, filter), built once.
struct FilterTable {
    float *H = nullptr;
    float2 *tw = nullptr;
    ~FilterTable() {
        if (H) (void)hipFree(H);
        if (tw) (void)hipFree(tw);
    }
};
static std::map<std::tuple<int, int, int>, std::unique_ptr<FilterTable>> g_filters;

static int filter_table(hipStream_t stream, int log2L, int filter, FilterTable **out) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return RADON_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_mutex);
    auto key = std::make_tuple(device, log2L, filter);
    auto it = g_filters.find(key);
    if (it != g_filters.end()) {
        *out = it->second.get();
        return RADON_OK;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return RADON_ERR_HIP;
    if (cap != hipStreamCaptureStatusNone) return RADON_ERR_NOT_PREPARED;
    std::vector<float> H;
    std::vector<float2> tw;
    filter_response(filter, log2L, H);
    filter_twiddles(log2L, tw);
    std::unique_ptr<FilterTable> t(new (std::nothrow) FilterTable());
    if (!t) return RADON_ERR_ALLOC;
    if (hipMalloc(&t->H, H.size() * sizeof(float)) != hipSuccess) return RADON_ERR_ALLOC;
    if (hipMalloc(&t->tw, tw.size() * sizeof(float2)) != hipSuccess) return RADON_ERR_ALLOC;
    if (hipMemcpy(t->H, H.data(), H.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
        return RADON_ERR_HIP;
    *out = t.get();
    g_filters.emplace(key, std::move(t));
    return RADON_OK;
}

// ---------------------------------------------------------------- uneven batches
// Device job/work tables of one uneven batch, built once per job list (by content:
// plans, buffers, batch sizes, scales) and reused, so later calls (and graph
// captures) only launch.  Every stream that launches a table gets its own work
// counter (slots of pooled blocks, so a capture stream takes one without
// allocating): launches of one job list on two streams never share a queue.
constexpr int kCounterSlots = 64;       // counters per block, 64 bytes apart
constexpr int kCounterStride = 16;      // ints between two counters
struct BatchTable {
    BatchJob *jobs = nullptr;
    ImageGroup *groups = nullptr;
    WorkUnit *work = nullptr;
    std::vector<int *> counter_blocks;
    std::map<hipStream_t, int *> counters;
    bool captured = false;       // launched under stream capture: a graph may replay it
    BatchLaunch launch;
    std::vector<int> fallback;   // jobs without a tiled plan, run with per-call kernels
    BatchTable() = default;
    BatchTable(const BatchTable &) = delete;
    BatchTable &operator=(const BatchTable &) = delete;
    ~BatchTable() {
        if (jobs) (void)hipFree(jobs);
        if (groups) (void)hipFree(groups);
        if (work) (void)hipFree(work);
        for (int *b : counter_blocks) (void)hipFree(b);
    }
};
static std::unordered_map<std::string, std::unique_ptr<BatchTable>> g_batches;
static std::deque<std::string> g_batch_order;
// tables dropped from the cache after a graph captured them: kept until
// radon_release_plans, since the graph may still replay them
static std::vector<std::unique_ptr<BatchTable>> g_batch_retired;
constexpr size_t kMaxBatchTables = 32;

static int alloc_counter_block(BatchTable &t) {
    int *b = nullptr;
    if (hipMalloc(&b, (size_t)kCounterSlots * kCounterStride * sizeof(int)) != hipSuccess)
        return RADON_ERR_ALLOC;
    t.counter_blocks.push_back(b);
    return RADON_OK;
}

// Work counter of table t for stream s (caller holds g_mutex).
static int stream_counter(BatchTable &t, hipStream_t s, bool capturing, int **out) {
    auto it = t.counters.find(s);
    if (it == t.counters.end()) {
        const size_t used = t.counters.size();
        if (used == t.counter_blocks.size() * kCounterSlots) {
            if (capturing) return RADON_ERR_NOT_PREPARED;
            const int rc = alloc_counter_block(t);
            if (rc != RADON_OK) return rc;
        }
        int *c = t.counter_blocks[used / kCounterSlots] + (used % kCounterSlots) * kCounterStride;
        it = t.counters.emplace(s, c).first;
    }
    *out = it->second;
    return RADON_OK;
}

template <typename V>
static int upload(V **dst, const std::vector<V> &src) {
    if (hipMalloc(dst, std::max<size_t>(src.size(), 1) * sizeof(V)) != hipSuccess) return RADON_ERR_ALLOC;
    if (!src.empty() &&
        hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice) != hipSuccess)
        return RADON_ERR_HIP;
    return RADON_OK;
}

// Images of all jobs that share a plan are pooled and cut into image groups, so
// single-image jobs of one geometry share lanes: forward, one 16-byte chunk of four
// images per lane (FP32 values or 16-bit tap pairs);
// backprojection, the narrowest of 8, 16 and 32 images that holds the images left (32
// while more remain).  Units are sorted longest first.
static int build_batch_table(const std::vector<Plan *> &plans, const radon_job_t *jobs, int n,
                             int dtype, int direction, int device, std::unique_ptr<BatchTable> &out) {
    std::unique_ptr<BatchTable> t(new (std::nothrow) BatchTable());
    if (!t) return RADON_ERR_ALLOC;
    const size_t esize = dtype == RADON_F32 ? 4 : 2;
    const int ch = dtype == RADON_F32 ? 4 : 8;
    struct Img { const char *in; char *out; float scale; };
    std::vector<Plan *> order;                       // distinct plans, first-seen order
    std::unordered_map<Plan *, std::vector<Img>> pool;
    for (int i = 0; i < n; ++i) {
        Plan *p = plans[i];
        if (jobs[i].batch == 0) continue;
        const bool tiled = direction == 0
                               ? (p->fwd_shape.variant == VARIANT_TILED && p->fwd_work[0].n_items > 0)
                               : (p->bp_shape.variant == VARIANT_TILED && p->bp_work.window > 0);
        if (!tiled) {
            t->fallback.push_back(i);
            continue;
        }
        const size_t img = (size_t)p->geom.n * p->geom.n * esize;
        const size_t sino = (size_t)p->geom.n_angles * p->geom.det_count * esize;
        const size_t in_stride = direction == 0 ? img : sino, out_stride = direction == 0 ? sino : img;
        if (!pool.count(p)) order.push_back(p);
        std::vector<Img> &v = pool[p];
        const float sdt = (float)(jobs[i].scale * jobs[i].geometry->step);
        for (int b = 0; b < jobs[i].batch; ++b)
            v.push_back({static_cast<const char *>(jobs[i].input) + b * in_stride,
                         static_cast<char *>(jobs[i].output) + b * out_stride, sdt});
    }
    std::vector<BatchJob> bj;
    std::vector<ImageGroup> groups;
    struct Unit { WorkUnit u; double cost; };
    std::vector<Unit> units;
    size_t lds = 16;
    for (Plan *p : order) {
        const std::vector<Img> &v = pool[p];
        BatchJob j{};
        j.g = p->geom;
        j.items = p->fwd_work[0].items;
        j.ranges = p->fwd_work[0].ranges;
        j.tile_t = p->fwd_work[0].tile_t;
        j.window = p->bp_work.window;
        j.bins = p->bp_work.bins;
        const int jid = (int)bj.size();
        bj.push_back(j);
        for (size_t k = 0; k < v.size();) {
            const size_t left = v.size() - k;
            const int cap = direction == 0 ? 4
                                           : (left > (size_t)kBatchBpMid    ? kBatchBpWide
                                              : left > (size_t)kBatchBpNarrow ? kBatchBpMid
                                                                              : kBatchBpNarrow);
            const int cnt = (int)std::min<size_t>(left, (size_t)cap);
            ImageGroup gr{};
            for (int e = 0; e < kBatchBpWide; ++e) {
                const Img &im = v[k + std::min(e, cnt - 1)];
                gr.in[e] = im.in;
                gr.out[e] = im.out;
                gr.scale[e] = im.scale;
            }
            gr.count = cnt;
            const int gid = (int)groups.size();
            groups.push_back(gr);
            k += cnt;
            if (direction == 0) {
                lds = std::max(lds, (size_t)(kSlabH + 3) * j.tile_t * sizeof(uint4));
                for (size_t it = 0; it < p->fwd_items_host.size(); ++it) {
                    const FwdItem &f = p->fwd_items_host[it];
                    units.push_back({{jid, (int)it, gid, 0}, (double)(f.nslab + 1) * f.na * f.nd});
                }
            } else {
                const int wide = cap == kBatchBpWide ? 1 : (cap == kBatchBpMid ? 2 : 0);
                const int planes = cap / ch;
                const int nimg = p->geom.n;
                const int tiles = ((nimg + kBpTile - 1) / kBpTile) * ((nimg + kBpTile - 1) / kBpTile);
                const size_t need = !p->geom.fan
                    ? (size_t)planes * kBpAngles * kBpWinPar * sizeof(uint4)
                    : (size_t)planes * kBpAnglesFan * j.window * sizeof(uint4) +
                          (size_t)kBpAnglesFan * j.window * sizeof(float4);
                lds = std::max(lds, need);
                // instruction estimate per (pixel, angle): candidate search + 3 or NB FMAs per image
                const int nb = p->geom.fan ? j.bins : 3;
                const double cost = (double)p->geom.n_angles * (30.0 * nb + cap * nb);
                for (int tile = 0; tile < tiles; ++tile)
                    units.push_back({{jid, tile, gid, wide}, cost});
            }
        }
    }
    std::stable_sort(units.begin(), units.end(),
                     [](const Unit &a, const Unit &b) { return a.cost > b.cost; });
    std::vector<WorkUnit> wu(units.size());
    for (size_t k = 0; k < units.size(); ++k) wu[k] = units[k].u;
    if (!bj.empty()) {
        int rc;
        if ((rc = upload(&t->jobs, bj)) != RADON_OK) return rc;
        if ((rc = upload(&t->groups, groups)) != RADON_OK) return rc;
        if ((rc = upload(&t->work, wu)) != RADON_OK) return rc;
        if ((rc = alloc_counter_block(*t)) != RADON_OK) return rc;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) return RADON_ERR_HIP;
        const int per_cu = batched_blocks_per_cu(direction, dtype, lds);
        t->launch.jobs = t->jobs;
        t->launch.groups = t->groups;
        t->launch.work = t->work;
        t->launch.n_work = (int)wu.size();
        t->launch.grid = std::max(1, std::min((int)wu.size(), per_cu * prop.multiProcessorCount));
        t->launch.lds = lds;
    }
    out = std::move(t);
    return RADON_OK;
}

static int run_batched(const radon_job_t *jobs, int32_t n, int32_t dtype, int direction,
                       void *stream) {
    int rc = check_dtype(dtype);
    if (rc != RADON_OK) return rc;
    if (n < 0 || (n > 0 && !jobs)) return RADON_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<Plan *> plans(n, nullptr);
    for (int i = 0; i < n; ++i) {
        const radon_job_t &j = jobs[i];
        if ((rc = validate(j.geometry)) != RADON_OK) return rc;
        if (j.batch < 0 || !std::isfinite(j.scale)) return RADON_ERR_INVALID_ARG;
        if (j.batch == 0) continue;
        if ((rc = check_ptr(j.input)) != RADON_OK || (rc = check_ptr(j.output)) != RADON_OK) return rc;
        if ((rc = get_plan(j.geometry, s, &plans[i])) != RADON_OK) return rc;
    }
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return RADON_ERR_NO_DEVICE;
    std::string key;
    key.reserve(16 + (size_t)n * 40);
    auto put = [&key](const void *p, size_t k) { key.append(static_cast<const char *>(p), k); };
    put(&device, sizeof device);
    put(&dtype, sizeof dtype);
    put(&direction, sizeof direction);
    for (int i = 0; i < n; ++i) {
        put(&plans[i], sizeof(Plan *));
        put(&jobs[i].input, sizeof(void *));
        put(&jobs[i].output, sizeof(void *));
        put(&jobs[i].batch, sizeof(int32_t));
        put(&jobs[i].scale, sizeof(float));
    }
    BatchTable *t = nullptr;
    BatchLaunch launch;
    {
        const bool capturing = is_capturing(s, &rc);
        if (rc != RADON_OK) return rc;
        std::lock_guard<std::mutex> lock(g_mutex);
        auto it = g_batches.find(key);
        if (it != g_batches.end()) {
            t = it->second.get();
        } else {
            if (capturing) return RADON_ERR_NOT_PREPARED;
            std::unique_ptr<BatchTable> nt;
            if ((rc = build_batch_table(plans, jobs, n, dtype, direction, device, nt)) != RADON_OK)
                return rc;
            if (g_batch_order.size() >= kMaxBatchTables) {
                auto old = g_batches.find(g_batch_order.front());
                if (old->second->captured) {
                    g_batch_retired.push_back(std::move(old->second));   // a graph may replay it
                } else {
                    (void)hipDeviceSynchronize();   // eager launches of it may still run
                }
                g_batches.erase(old);
                g_batch_order.pop_front();
            }
            t = nt.get();
            g_batches.emplace(key, std::move(nt));
            g_batch_order.push_back(key);
        }
        launch = t->launch;
        if (launch.n_work > 0 && (rc = stream_counter(*t, s, capturing, &launch.counter)) != RADON_OK)
            return rc;
        t->captured = t->captured || capturing;
    }
    if (launch.n_work > 0) {
        hipError_t e = launch_batched(direction, dtype, launch, s);
        if (e != hipSuccess) return RADON_ERR_HIP;
    }
    for (int i : t->fallback) {
        const Plan *p = plans[i];
        hipError_t e = direction == 0
            ? launch_forward(p->geom, p->fwd_work[0], dtype, p->fwd_shape, jobs[i].input,
                             jobs[i].output, jobs[i].batch, jobs[i].scale, nullptr, 0, s)
            : launch_backproject(p->geom, p->bp_work, dtype, p->bp_shape, jobs[i].input,
                                 jobs[i].output, jobs[i].batch, jobs[i].scale, nullptr, 0, s);
        if (e != hipSuccess) return RADON_ERR_HIP;
    }
    return RADON_OK;
}

static int release_all() {
    std::lock_guard<std::mutex> lock(g_mutex);
    (void)hipDeviceSynchronize();
    release_shearlet_plans();
    g_batches.clear();
    g_batch_order.clear();
    g_batch_retired.clear();
    g_plans.clear();
    g_filters.clear();
    for (auto &kv : g_workspaces) {
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        for (void *r : kv.second.retired) (void)hipFree(r);
    }
    g_workspaces.clear();
    for (auto &kv : g_scratch) {
        for (double *b : kv.second.dot_blocks) (void)hipFree(b);
        for (void *r : kv.second.retired) (void)hipFree(r);
    }
    for (auto &kv : g_stream_scratch)
        if (kv.second.row_partials) (void)hipFree(kv.second.row_partials);
    g_scratch.clear();
    g_stream_scratch.clear();
    return RADON_OK;
}

// The forward tiling t if its plan exists, else tiling 0.
static void use_tiling(const Plan *p, LaunchShape &fwd, int t) {
    fwd.tiling = (t >= 0 && t < kFwdTilings && p->fwd_work[t].n_items > 0) ? t : 0;
    fwd.angles = kFwdTiling[fwd.tiling].waves;
}

// Launch shapes for a call: the autotuned ones for this storage type and batch class
// when radon_prepare has tuned them, else the plan's defaults.
// RADON_FORCE_SHAPE="fi,fs,bi,ba[,bs[,ft]]" overrides both (used to test every variant).
static void call_shapes(Plan *p, int dtype, int batch, LaunchShape &fwd, LaunchShape &bp) {
    fwd = p->fwd_shape;
    bp = p->bp_shape;
    // test hook: "fwd images, fwd staging, bp images, bp angles[, bp staging[, fwd tiling]]"
    if (const char *f = std::getenv("RADON_FORCE_SHAPE")) {
        int fi, fs, bi, ba, bs = 1, ft = 0;
        const int k = std::sscanf(f, "%d,%d,%d,%d,%d,%d", &fi, &fs, &bi, &ba, &bs, &ft);
        if (k >= 4) {
            fwd.images = fi;
            fwd.stage = fs;
            use_tiling(p, fwd, ft);
            bp.images = bi;
            bp.angles = p->geom.fan ? (ba == 2 ? 2 : kBpAnglesFan) : ba;
            bp.stage = bs;
            return;
        }
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    auto it = p->tuned.find({dtype, batch_class(batch)});
    if (it == p->tuned.end() || !it->second.valid) {
        // untuned small batches: the narrowest tiled shapes leave the fewest lanes
        // without an image (one 16-byte chunk per lane: 4 FP32 or 8 16-bit images)
        const int chunk = dtype == F32 ? 4 : 8;
        if (fwd.variant == VARIANT_TILED && dtype == F32 && batch <= 4) fwd.images = 4;
        if (bp.variant == VARIANT_TILED && batch <= 16) bp.images = batch <= chunk ? 4 : 16;
        if (bp.variant == VARIANT_TILED && batch <= chunk) bp.stage = 0;   // no copy for one chunk
        return;
    }
    fwd.variant = it->second.fwd_variant;
    bp.variant = it->second.bp_variant;
    fwd.images = it->second.fwd_images;
    fwd.stage = it->second.fwd_stage;
    use_tiling(p, fwd, it->second.fwd_tiling);
    bp.images = it->second.bp_images;
    bp.angles = it->second.bp_angles;
    bp.stage = it->second.bp_stage;
}

}  // namespace radon

using namespace radon;

extern "C" {

int radon_validate(const radon_geometry_t *geometry) { return validate(geometry); }

int radon_prepare(const radon_geometry_t *geometry, int32_t dtype, int32_t batch) {
    int rc = validate(geometry);
    if (rc != RADON_OK) return rc;
    if ((rc = check_dtype(dtype)) != RADON_OK) return rc;
    if (batch < 0) return RADON_ERR_INVALID_ARG;
    Plan *p = nullptr;
    rc = get_plan(geometry, nullptr, &p);
    if (rc != RADON_OK) return rc;
    const char *tune = std::getenv("RADON_AUTOTUNE");
    const bool want = !(tune && std::strcmp(tune, "0") == 0);
    if (want && batch > 0) {
        bool have;
        {
            std::lock_guard<std::mutex> lock(g_mutex);
            auto it = p->tuned.find({dtype, batch_class(batch)});
            have = it != p->tuned.end() && it->second.valid;
        }
        if (!have) {
            size_t ws_bytes = 0;
            const size_t need = std::max(
                interleaved_bytes(geometry->image_size, batch, dtype),
                interleaved_sino_bytes(p->geom.n_angles, p->geom.det_count, p->bp_work.window, batch, dtype));
            void *ws = stream_workspace(nullptr, need, &ws_bytes);
            TunedShapes t;
            if (autotune(*p, dtype, batch, ws, ws_bytes, t) == 0) {
                std::lock_guard<std::mutex> lock(g_mutex);
                p->tuned[{dtype, batch_class(batch)}] = t;
            }
        }
    }
    return hipDeviceSynchronize() == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_forward(const radon_geometry_t *geometry, const void *x, void *y, int32_t batch,
                  int32_t dtype, float scale, void *stream) {
    int rc = validate(geometry);
    if (rc != RADON_OK) return rc;
    if ((rc = check_dtype(dtype)) != RADON_OK) return rc;
    if (batch < 0 || !std::isfinite(scale)) return RADON_ERR_INVALID_ARG;
    if (batch == 0) return RADON_OK;
    if ((rc = check_ptr(x)) != RADON_OK || (rc = check_ptr(y)) != RADON_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Plan *p = nullptr;
    if ((rc = get_plan(geometry, s, &p)) != RADON_OK) return rc;
    LaunchShape fwd, bp;
    call_shapes(p, dtype, batch, fwd, bp);
    void *ws = nullptr;
    size_t ws_bytes = 0;
    if (fwd.variant == VARIANT_TILED && fwd.stage && p->fwd_work[fwd.tiling].n_items > 0 && !p->no_interleave)
        ws = stream_workspace(s, interleaved_bytes(geometry->image_size, batch, dtype), &ws_bytes);
    hipError_t e = launch_forward(p->geom, p->fwd_work[fwd.tiling], dtype, fwd, x, y, batch, scale, ws,
                                  ws_bytes, s);
    return e == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_backproject(const radon_geometry_t *geometry, const void *y, void *x, int32_t batch,
                      int32_t dtype, float scale, void *stream) {
    int rc = validate(geometry);
    if (rc != RADON_OK) return rc;
    if ((rc = check_dtype(dtype)) != RADON_OK) return rc;
    if (batch < 0 || !std::isfinite(scale)) return RADON_ERR_INVALID_ARG;
    if (batch == 0) return RADON_OK;
    if ((rc = check_ptr(x)) != RADON_OK || (rc = check_ptr(y)) != RADON_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Plan *p = nullptr;
    if ((rc = get_plan(geometry, s, &p)) != RADON_OK) return rc;
    LaunchShape fwd, bp;
    call_shapes(p, dtype, batch, fwd, bp);
    void *ws = nullptr;
    size_t ws_bytes = 0;
    if (bp.variant == VARIANT_TILED && bp.stage && p->bp_work.window > 0)
        ws = stream_workspace(s, interleaved_sino_bytes(p->geom.n_angles, p->geom.det_count,
                                                        p->bp_work.window, batch, dtype),
                              &ws_bytes);
    hipError_t e = launch_backproject(p->geom, p->bp_work, dtype, bp, y, x, batch, scale, ws,
                                      ws_bytes, s);
    return e == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_forward_batched(const radon_job_t *jobs, int32_t n_jobs, int32_t dtype, void *stream) {
    return run_batched(jobs, n_jobs, dtype, 0, stream);
}

int radon_backproject_batched(const radon_job_t *jobs, int32_t n_jobs, int32_t dtype,
                              void *stream) {
    return run_batched(jobs, n_jobs, dtype, 1, stream);
}

int radon_filter_sinogram(const radon_geometry_t *geometry, const void *y, void *out,
                          int32_t batch, int32_t filter, int32_t dtype, void *stream) {
    int rc = validate(geometry);
    if (rc != RADON_OK) return rc;
    if ((rc = check_dtype(dtype)) != RADON_OK) return rc;
    if (filter < FILTER_RAMLAK || filter > FILTER_HANN || batch < 0) return RADON_ERR_INVALID_ARG;
    if (geometry->beam != RADON_PARALLEL) return RADON_ERR_UNSUPPORTED;
    const int log2L = filter_log2_length(geometry->det_count);
    if (log2L > kFilterMaxLog2) return RADON_ERR_UNSUPPORTED;
    if (batch == 0) return RADON_OK;
    if ((rc = check_ptr(y)) != RADON_OK || (rc = check_ptr(out)) != RADON_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    FilterTable *t = nullptr;
    if ((rc = filter_table(s, log2L, filter, &t)) != RADON_OK) return rc;
    // pi / A: the sampled kernel's 1/spacing cancels against the 1/spacing density of
    // bins that the exact transpose gathers per unit of detector length
    const double pi = 3.14159265358979323846;
    const float scale = (float)(pi / (double)geometry->n_angles);
    const long long rows = (long long)batch * geometry->n_angles;
    hipError_t e = launch_filter(dtype, y, out, rows, geometry->det_count, log2L, t->H, t->tw,
                                 scale, s);
    return e == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_dot_f64(const void *a, const void *b, int64_t n, int32_t dtype, double *out,
                  void *stream) {
    int rc = check_dtype(dtype);
    if (rc != RADON_OK) return rc;
    if (n < 0) return RADON_ERR_INVALID_ARG;
    if (!out) return RADON_ERR_INVALID_ARG;
    if (n > 0 && ((rc = check_ptr(a)) != RADON_OK || (rc = check_ptr(b)) != RADON_OK)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *partials = nullptr;
    if ((rc = dot_scratch(s, &partials)) != RADON_OK) return rc;
    hipError_t e = launch_dot_f64(a, b, (long long)n, dtype, out, partials, kDotPartials, s);
    return e == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_dot_f64_batched(const void *a, const void *b, int64_t n, int32_t batch, int32_t dtype,
                          double *out, void *stream) {
    int rc = check_dtype(dtype);
    if (rc != RADON_OK) return rc;
    if (n < 0 || batch < 0 || batch > 65535 || !out) return RADON_ERR_INVALID_ARG;
    if (batch == 0) return RADON_OK;
    if (reinterpret_cast<uintptr_t>(out) % alignof(double)) return RADON_ERR_ALIGN;
    if (n > 0 && ((rc = check_ptr(a)) != RADON_OK || (rc = check_ptr(b)) != RADON_OK)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *partials = nullptr;
    if ((rc = row_scratch(s, (size_t)batch * dot_rows_chunks(n), &partials)) != RADON_OK) return rc;
    hipError_t e = launch_dot_rows(a, b, (long long)n, batch, dtype, out, partials, s);
    return e == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_dot_f64_batched_noalloc(const void *a, const void *b, int64_t n, int32_t batch,
                                  int32_t dtype, double *out, void *stream) {
    int rc = check_dtype(dtype);
    if (rc != RADON_OK) return rc;
    if (n < 0 || batch < 0 || batch > 65535 || !out) return RADON_ERR_INVALID_ARG;
    if (batch == 0) return RADON_OK;
    if (reinterpret_cast<uintptr_t>(out) % alignof(double)) return RADON_ERR_ALIGN;
    if (n > 0 && ((rc = check_ptr(a)) != RADON_OK || (rc = check_ptr(b)) != RADON_OK)) return rc;
    if ((long long)batch * dot_rows_chunks(n) > kStaticDotPartials) return RADON_ERR_SCRATCH;
    double *partials = nullptr;
    if (static_dot_partials(&partials) != hipSuccess) return RADON_ERR_HIP;
    hipError_t e = launch_dot_rows(a, b, (long long)n, batch, dtype, out, partials,
                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_axpy_ratio(const void *u, const void *v, void *out, const double *num,
                     const double *den, double c0, int64_t n, int32_t batch, int32_t dtype,
                     void *stream) {
    int rc = check_dtype(dtype);
    if (rc != RADON_OK) return rc;
    if (n < 0 || batch < 0 || batch > 65535 || !std::isfinite(c0)) return RADON_ERR_INVALID_ARG;
    if (n == 0 || batch == 0) return RADON_OK;
    if ((rc = check_ptr(u)) != RADON_OK || (rc = check_ptr(v)) != RADON_OK ||
        (rc = check_ptr(out)) != RADON_OK)
        return rc;
    if (reinterpret_cast<uintptr_t>(num) % alignof(double) ||
        reinterpret_cast<uintptr_t>(den) % alignof(double))
        return RADON_ERR_ALIGN;
    hipError_t e = launch_axpy_ratio(u, v, out, num, den, c0, (long long)n, batch, dtype,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_release_plans(void) { return release_all(); }

int radon_plan_info(const radon_geometry_t *geometry, int32_t dtype, int32_t batch,
                    int32_t *out10) {
    int rc = validate(geometry);
    if (rc != RADON_OK) return rc;
    if ((rc = check_dtype(dtype)) != RADON_OK) return rc;
    if (!out10 || batch < 0) return RADON_ERR_INVALID_ARG;
    Plan *p = nullptr;
    if ((rc = get_plan(geometry, nullptr, &p)) != RADON_OK) return rc;
    LaunchShape fwd, bp;
    call_shapes(p, dtype, std::max(batch, 1), fwd, bp);
    if (bp.variant != VARIANT_TILED) bp.stage = 0;
    if (fwd.variant != VARIANT_TILED || p->no_interleave) fwd.stage = 0;
    const LaunchShape *sh[2] = {&fwd, &bp};
    for (int i = 0; i < 2; ++i) {
        out10[5 * i + 0] = sh[i]->images;
        out10[5 * i + 1] = sh[i]->angles;
        out10[5 * i + 2] = sh[i]->stage;
        out10[5 * i + 3] = sh[i]->variant;
    }
    out10[4] = kFwdTiling[fwd.tiling].slab_h;
    out10[9] = kBpTile;
    return RADON_OK;
}

const char *radon_status_string(int status) {
    switch (status) {
    case RADON_OK: return "ok";
    case RADON_ERR_INVALID_ARG: return "invalid argument";
    case RADON_ERR_ALIGN: return "device pointer not 16-byte aligned";
    case RADON_ERR_UNSUPPORTED: return "unsupported request";
    case RADON_ERR_HIP: return "HIP runtime error";
    case RADON_ERR_ALLOC: return "allocation failed";
    case RADON_ERR_NO_DEVICE: return "no usable GPU";
    case RADON_ERR_NOT_PREPARED: return "plan missing while the stream is capturing";
    case RADON_ERR_SCRATCH: return "request exceeds the fixed scratch of a no-allocation entry point";
    default: return "unknown status";
    }
}

int radon_version(void) { return 100; }

}  // extern "C"
