// Autotuner: picks the launch shape of each direction for a (plan, storage type,
// batch size class) by timing the candidates on the device with HIP events.
//
// Forward candidates: images per lane {8, 16, 4 (FP32 only)} x slab
// staging {interleaved copy, caller's images, and for 16-bit storage the tap-pair copy
// with dot2 arithmetic} x tiling (kFwdTiling: slab rows {11, 7, 15} with 8 angles per
// work item, and 11 rows with 4 angles), and the direct kernel.
// Backprojection candidates: images per lane {64, 32, 16, one chunk (batches <= 8)} x
// angles per LDS block (with the interleaved copies, whose next block is copied
// asynchronously into a second buffer, {4, 2}; from the caller's sinograms {8, 4}
// parallel, 4 fan) x sinogram staging {interleaved copy, caller's sinograms, and for 16-bit storage
// the tap-pair copy with dot2 arithmetic}, and the direct kernel.  Every candidate is
// timed once (a warm-up launch, then three), the three fastest three more times
// round-robin, and the fastest timing decides.  The direct kernels win on tiny problems, where the
// tiled kernels' sequential slabs and angle blocks are latency-bound.  Results live in the plan
// and, when RADON_TUNE_CACHE names a file, in that file (one line per entry:
// "<key> <fwd variant> <fwd images> <fwd stage> <bp variant> <bp images> <bp angles>
// <bp stage> <fwd tiling>"),
// so later processes skip the timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "radon_autotune.hpp"

namespace radon {

int batch_class(int batch) {
    int c = 1;
    while (c < batch && c < (1 << 20)) c <<= 1;
    return c;
}

static std::string tune_key(const Plan &p, int dtype, int bclass) {
    std::ostringstream k;
    k << "g" << std::hex << p.key_hash << std::dec << "_n" << p.geom.n << "_a" << p.geom.n_angles
      << "_d" << p.geom.det_count << "_f" << p.geom.fan << "_t" << dtype << "_b" << bclass;
    return k.str();
}

static bool cache_lookup(const std::string &key, TunedShapes &out) {
    const char *path = std::getenv("RADON_TUNE_CACHE");
    if (!path || !*path) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream ls(line);
        std::string k;
        int fv, fi, fs, bv, bi, ba, bs, ft = 0;
        if (!(ls >> k >> fv >> fi >> fs >> bv >> bi >> ba >> bs) || k != key) continue;
        if (!(ls >> ft) || ft < 0 || ft >= kFwdTilings) ft = 0;   // lines of older versions: tiling 0
        out.fwd_variant = fv;
        out.bp_variant = bv;
        out.fwd_images = fi;
        out.fwd_stage = fs;
        out.bp_images = bi;
        out.bp_angles = ba;
        out.bp_stage = bs;
        out.fwd_tiling = ft;
        return true;
    }
    return false;
}

static void cache_store(const std::string &key, const TunedShapes &t) {
    const char *path = std::getenv("RADON_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << t.fwd_variant << " " << t.fwd_images << " " << t.fwd_stage << " "
      << t.bp_variant << " " << t.bp_images << " " << t.bp_angles << " " << t.bp_stage << " "
      << t.fwd_tiling << "\n";
}

// Average milliseconds of `reps` launches after one warm-up; a negative value when
// a launch fails.
template <class F>
static float time_launches(F launch, hipStream_t s, int reps = 3) {
    if (launch() != hipSuccess) return -1.0f;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1.0f;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return -1.0f; }
    float ms = -1.0f;
    bool ok = hipEventRecord(a, s) == hipSuccess;
    for (int i = 0; ok && i < reps; ++i) ok = launch() == hipSuccess;
    ok = ok && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
         hipEventElapsedTime(&ms, a, b) == hipSuccess;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ok ? ms / reps : -1.0f;
}

// The candidates within a few percent of each other after one timing each can swap
// places between runs (launch-to-launch jitter, clocks), so the three fastest are timed
// again, round-robin, three more times each, and the fastest of every candidate's
// timings wins.  Returns the index of the winner in `ms` (or -1 if none ran).
template <class F>
static int pick_fastest(std::vector<float> &ms, F time_candidate) {
    std::vector<int> order;
    for (int i = 0; i < (int)ms.size(); ++i)
        if (ms[i] > 0.0f) order.push_back(i);
    if (order.empty()) return -1;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return ms[a] < ms[b]; });
    if (order.size() > 3) order.resize(3);
    for (int round = 0; round < 3; ++round)
        for (int i : order) {
            const float t = time_candidate(i);
            if (t > 0.0f && t < ms[i]) ms[i] = t;
        }
    int best = order[0];
    for (int i : order)
        if (ms[i] < ms[best]) best = i;
    return best;
}

int autotune(Plan &p, int dtype, int batch, void *ws, size_t ws_bytes, TunedShapes &out) {
    const int bclass = batch_class(batch);
    const std::string key = tune_key(p, dtype, bclass);
    out = TunedShapes{};
    out.fwd_images = p.fwd_shape.images;
    out.fwd_stage = p.fwd_shape.stage;
    out.bp_images = p.bp_shape.images;
    out.bp_angles = p.bp_shape.angles;
    out.bp_stage = p.bp_shape.stage;
    out.fwd_variant = p.fwd_shape.variant;
    out.bp_variant = p.bp_shape.variant;
    if (cache_lookup(key, out)) {
        out.valid = true;
        return 0;
    }
    const size_t es = dtype == F32 ? 4 : 2;
    const size_t xb = (size_t)batch * p.geom.n * p.geom.n * es;
    const size_t yb = (size_t)batch * p.geom.n_angles * p.geom.det_count * es;
    void *x = nullptr, *y = nullptr;
    if (hipMalloc(&x, std::max<size_t>(xb, 16)) != hipSuccess) return -1;
    if (hipMalloc(&y, std::max<size_t>(yb, 16)) != hipSuccess) { (void)hipFree(x); return -1; }
    hipStream_t s = nullptr;
    // data-like inputs: the kernels' speed depends on the data (power), and zeros
    // favour shapes that lose on real images
    if (launch_fill_pattern(x, (long long)(xb / es), dtype, 1u, s) != hipSuccess ||
        launch_fill_pattern(y, (long long)(yb / es), dtype, 2u, s) != hipSuccess) {
        (void)hipFree(x);
        (void)hipFree(y);
        return -1;
    }

    if (p.fwd_shape.variant == VARIANT_TILED) {
        std::vector<int> imgs = dtype == F32 ? std::vector<int>{8, 4, 16} : std::vector<int>{8, 16};
        // candidate 0: the direct kernel; then tilings x images x staging
        std::vector<LaunchShape> cands;
        LaunchShape direct = p.fwd_shape;
        direct.variant = VARIANT_DIRECT;
        cands.push_back(direct);
        const std::vector<int> stages = dtype == F32 ? std::vector<int>{1, 0} : std::vector<int>{2, 1, 0};
        for (int t = 0; t < kFwdTilings; ++t) {
            if (p.fwd_work[t].n_items == 0) continue;
            for (int im : imgs)
                for (int st : stages) {
                    if (st > 0 && p.no_interleave) continue;
                    LaunchShape sh = p.fwd_shape;
                    sh.images = im;
                    sh.stage = st;
                    sh.tiling = t;
                    cands.push_back(sh);
                }
        }
        auto time_fwd = [&](int i) {
            const LaunchShape &sh = cands[i];
            const FwdWork &w = p.fwd_work[sh.variant == VARIANT_DIRECT ? 0 : sh.tiling];
            return time_launches([&] {
                return launch_forward(p.geom, w, dtype, sh, x, y, batch, 1.0f, ws, ws_bytes, s);
            }, s);
        };
        std::vector<float> ms(cands.size());
        for (int i = 0; i < (int)cands.size(); ++i) ms[i] = time_fwd(i);
        const int b = pick_fastest(ms, time_fwd);
        out.fwd_variant = VARIANT_DIRECT;
        if (b > 0) {
            out.fwd_variant = VARIANT_TILED;
            out.fwd_images = cands[b].images;
            out.fwd_stage = cands[b].stage;
            out.fwd_tiling = cands[b].tiling;
        }
    }
    if (p.bp_shape.variant == VARIANT_TILED) {
        std::vector<LaunchShape> cands;
        LaunchShape direct = p.bp_shape;
        direct.variant = VARIANT_DIRECT;
        cands.push_back(direct);
        // angles per LDS block: the double-buffered kernels on the interleaved copies
        // (stages 1, 2) take {4, 2}, the caller's sinograms (stage 0) the parallel
        // beam's {8, 4} and the fan beam's 4
        auto abs = [&](int st) {
            if (st > 0) return std::vector<int>{4, 2};
            return p.geom.fan ? std::vector<int>{kBpAnglesFan} : std::vector<int>{kBpAngles, 4};
        };
        // one chunk per lane (4 FP32 or 8 16-bit images) only pays for small batches
        const std::vector<int> ims{64, 32, 16, 4};
        for (int im : ims)
            if (im >= 16 || batch <= 8)
            for (int st : (dtype == F32 ? std::vector<int>{1, 0} : std::vector<int>{2, 1, 0}))
                for (int ab : abs(st)) {
                    LaunchShape sh = p.bp_shape;
                    sh.images = im;
                    sh.angles = ab;
                    sh.stage = st;
                    cands.push_back(sh);
                }
        auto time_bp = [&](int i) {
            return time_launches([&] {
                return launch_backproject(p.geom, p.bp_work, dtype, cands[i], y, x, batch, 1.0f, ws, ws_bytes, s);
            }, s);
        };
        std::vector<float> ms(cands.size());
        for (int i = 0; i < (int)cands.size(); ++i) ms[i] = time_bp(i);
        const int b = pick_fastest(ms, time_bp);
        out.bp_variant = VARIANT_DIRECT;
        if (b > 0) {
            out.bp_variant = VARIANT_TILED;
            out.bp_images = cands[b].images;
            out.bp_angles = cands[b].angles;
            out.bp_stage = cands[b].stage;
        }
    }
    (void)hipDeviceSynchronize();
    (void)hipFree(x);
    (void)hipFree(y);
    out.valid = true;
    cache_store(key, out);
    return 0;
}

}  // namespace radon
