// CPU check of the library's kernels, built against the host emulation of HIP with
// AddressSanitizer.  For every geometry of a list it runs the per-call forward and
// backprojection (tiled kernels where the planner accepts the geometry), the direct
// kernels, and the FP64 oracle on the same inputs, and reports the relative L2
// differences; with "batched" it also runs the whole list as one uneven batch in each
// direction and compares it with the per-call results bitwise.
//
// Line format: beam n D spacing S E step batch dtype A angle_0 ... angle_{A-1}
// Output: one "geometry ..." line per geometry, then "batched ..." and "summary ...".
// The "filter" and "solver" modes write their results to a file instead.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <random>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "radon.h"

extern "C" {
int oracle_forward(int beam, int n, int n_angles, const double *angles, int det_count,
                   double det_spacing, double source_distance, double det_distance, double step,
                   const double *x, int batch, double scale, double *y);
int oracle_backproject(int beam, int n, int n_angles, const double *angles, int det_count,
                       double det_spacing, double source_distance, double det_distance,
                       double step, const double *y, int batch, double scale, double *x);
}

namespace {

struct Geo {
    int beam, n, D, batch, dt, A;
    double sp, S, E, step;
    std::vector<double> angles;
    radon_geometry_t g;
    size_t nx, ny;
    std::vector<unsigned char> x, y;           // inputs (storage type)
    void *fx = nullptr, *bx = nullptr;         // per-call outputs
    std::vector<double> oracle_fx;             // FP64 oracle forward on the stored inputs
};

size_t esize(int dt) { return dt == RADON_F32 ? 4 : 2; }

double to_double(const void *p, size_t i, int dt) {
    if (dt == RADON_F32) return ((const float *)p)[i];
    const unsigned short h = ((const unsigned short *)p)[i];
    if (dt == RADON_BF16) {
        const unsigned u = (unsigned)h << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    }
    _Float16 f;
    std::memcpy(&f, &h, 2);
    return (float)f;
}

void from_float(void *p, size_t i, float v, int dt) {
    if (dt == RADON_F32) { ((float *)p)[i] = v; return; }
    if (dt == RADON_BF16) {      // round to nearest even
        unsigned u;
        std::memcpy(&u, &v, 4);
        u += 0x7fffu + ((u >> 16) & 1u);
        ((unsigned short *)p)[i] = (unsigned short)(u >> 16);
        return;
    }
    const _Float16 h = (_Float16)v;
    std::memcpy((unsigned short *)p + i, &h, 2);
}

double rel_l2(const void *a, int dt, const double *ref, size_t n) {
    double num = 0.0, den = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const double d = to_double(a, i, dt) - ref[i];
        num += d * d;
        den += ref[i] * ref[i];
    }
    return den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
}

void *dev_alloc(size_t bytes) {
    void *p = nullptr;
    if (posix_memalign(&p, 256, bytes ? bytes : 1) != 0) return nullptr;
    return p;
}

}  // namespace

// "filter" mode: for every geometry, radon_filter_sinogram with each of the five
// filters on the geometry's random sinograms; writes, per geometry, the input and the
// five outputs (as FP64) to the file named by argv[3].
static int filter_mode(std::vector<Geo> &geos, const char *path) {
    FILE *out = std::fopen(path, "wb");
    if (!out) return 2;
    int fails = 0;
    for (size_t k = 0; k < geos.size(); ++k) {
        Geo &g = geos[k];
        const size_t es = esize(g.dt);
        void *yin = dev_alloc(g.ny * es), *yo = dev_alloc(g.ny * es);
        std::memcpy(yin, g.y.data(), g.ny * es);
        std::vector<double> buf(g.ny);
        for (size_t i = 0; i < g.ny; ++i) buf[i] = to_double(g.y.data(), i, g.dt);
        std::fwrite(buf.data(), sizeof(double), g.ny, out);
        for (int f = 0; f < 5; ++f) {
            std::fprintf(stderr, "[emu] filter %d geometry %zu\n", f, k);
            const int rc = radon_filter_sinogram(&g.g, yin, yo, g.batch, f, g.dt, nullptr);
            if (rc) {
                std::printf("geometry %zu filter %d status %d\n", k, f, rc);
                ++fails;
            }
            for (size_t i = 0; i < g.ny; ++i) buf[i] = rc ? 0.0 : to_double(yo, i, g.dt);
            std::fwrite(buf.data(), sizeof(double), g.ny, out);
        }
        std::free(yin);
        std::free(yo);
    }
    std::fclose(out);
    std::printf("summary geometries %zu failures %d\n", geos.size(), fails);
    return fails ? 1 : 0;
}

// "solver" mode: for every geometry, `iters` steps of radon_landweber (step alpha) and
// of radon_cgne from the geometry's random image x towards its random sinogram y, and
// the per-system inner products <x, x>; writes, per geometry, x, y, the Landweber
// result, the CGNE result (FP64) and the batch inner products to argv[3].
static int solver_mode(std::vector<Geo> &geos, const char *path, double alpha, int iters) {
    FILE *out = std::fopen(path, "wb");
    if (!out) return 2;
    int fails = 0;
    for (size_t k = 0; k < geos.size(); ++k) {
        Geo &g = geos[k];
        const size_t es = esize(g.dt);
        void *x = dev_alloc(g.nx * es), *y = dev_alloc(g.ny * es), *dots = dev_alloc(g.batch * 8);
        std::vector<double> buf(std::max(g.nx, g.ny));
        auto dump = [&](const void *p, size_t n) {
            for (size_t i = 0; i < n; ++i) buf[i] = to_double(p, i, g.dt);
            std::fwrite(buf.data(), sizeof(double), n, out);
        };
        dump(g.x.data(), g.nx);
        dump(g.y.data(), g.ny);
        std::memcpy(y, g.y.data(), g.ny * es);
        int rc = 0;
        for (int solver = 0; solver < 2; ++solver) {
            std::fprintf(stderr, "[emu] solver %d geometry %zu\n", solver, k);
            std::memcpy(x, g.x.data(), g.nx * es);
            const int64_t bytes = radon_solver_workspace_bytes(&g.g, solver, g.batch, g.dt);
            void *ws = bytes > 0 ? dev_alloc((size_t)bytes) : nullptr;
            rc = bytes < 0 ? (int)bytes
                 : solver == RADON_SOLVER_LANDWEBER
                     ? radon_landweber(&g.g, y, x, g.batch, alpha, iters, g.dt, ws, bytes, nullptr)
                     : radon_cgne(&g.g, y, x, g.batch, iters, g.dt, ws, bytes, nullptr);
            std::free(ws);
            if (rc) {
                std::printf("geometry %zu solver %d status %d\n", k, solver, rc);
                ++fails;
            }
            dump(x, g.nx);
        }
        std::memcpy(x, g.x.data(), g.nx * es);
        rc = radon_dot_f64_batched(x, x, (int64_t)g.n * g.n, g.batch, g.dt, (double *)dots, nullptr);
        if (rc) {
            std::printf("geometry %zu dot status %d\n", k, rc);
            ++fails;
        }
        std::fwrite(dots, sizeof(double), g.batch, out);
        std::free(x);
        std::free(y);
        std::free(dots);
    }
    std::fclose(out);
    std::printf("summary geometries %zu failures %d\n", geos.size(), fails);
    return fails ? 1 : 0;
}

// "lifetime" mode: graph-capture lifetime and stream separation.  The geometries form
// one job list L0 (forward).  L0 runs eagerly on stream A, then is captured on A and
// on B; the two captured persistent launches must differ in their arguments (each
// stream has its own work counter).  Forty more job lists (fresh output buffers) then
// push L0's table out of the cache; replaying the captured launches afterwards must
// still reproduce the eager outputs bitwise (AddressSanitizer reports a freed table),
// also with A's and B's replays running at the same time.  The FP64 inner product is
// captured on A and B the same way.  No allocation may happen while a stream captures.
static int lifetime_mode(std::vector<Geo> &geos) {
    hipStream_t A = reinterpret_cast<hipStream_t>(0x1000), B = reinterpret_cast<hipStream_t>(0x2000);
    const int dt = geos[0].dt;
    const size_t es = esize(dt);
    std::vector<radon_job_t> l0;
    std::vector<void *> outs, eager, keep;
    for (Geo &g : geos) {
        void *xin = dev_alloc(g.nx * es);
        std::memcpy(xin, g.x.data(), g.nx * es);
        keep.push_back(xin);
        outs.push_back(dev_alloc(g.ny * es));
        eager.push_back(dev_alloc(g.ny * es));
        l0.push_back(radon_job_t{&g.g, xin, outs.back(), g.batch, 1.0f});
    }
    int fails = 0;
    auto expect = [&](bool ok, const char *what) {
        std::printf("check %s %s\n", what, ok ? "ok" : "FAILED");
        fails += !ok;
    };
    const int n = (int)l0.size();
    int rc = radon_forward_batched(l0.data(), n, dt, A);
    expect(rc == 0, "eager_status");
    for (int k = 0; k < n; ++k) std::memcpy(eager[k], outs[k], geos[k].ny * es);
    emu::begin_capture(A);
    rc = radon_forward_batched(l0.data(), n, dt, A);
    auto graph_a = emu::end_capture(A);
    emu::begin_capture(B);
    const int rc_b = radon_forward_batched(l0.data(), n, dt, B);
    auto graph_b = emu::end_capture(B);
    expect(rc == 0 && rc_b == 0 && !graph_a.empty() && graph_a.size() == graph_b.size(),
           "capture_status");
    bool differ = false;
    for (size_t i = 0; i < graph_a.size() && i < graph_b.size(); ++i)
        differ = differ || graph_a[i].args != graph_b[i].args;
    expect(differ, "streams_use_own_counters");
    // forty more job lists evict L0's table from the cache
    for (int list = 0; list < 40; ++list) {
        std::vector<radon_job_t> li = l0;
        for (int k = 0; k < n; ++k) {
            li[k].output = dev_alloc(geos[k].ny * es);
            keep.push_back(li[k].output);
        }
        if (radon_forward_batched(li.data(), n, dt, A) != 0) {
            expect(false, "eviction_lists");
            break;
        }
    }
    auto same = [&]() {
        bool ok = true;
        for (int k = 0; k < n; ++k) ok = ok && std::memcmp(outs[k], eager[k], geos[k].ny * es) == 0;
        return ok;
    };
    auto poison = [&]() {
        for (int k = 0; k < n; ++k) std::memset(outs[k], 0xff, geos[k].ny * es);
    };
    poison();
    emu::replay_graph(graph_a);
    expect(same(), "replay_after_eviction");
    poison();
    std::thread ta([&] { emu::replay_graph(graph_a); });
    std::thread tb([&] { emu::replay_graph(graph_b); });
    ta.join();
    tb.join();
    expect(same(), "concurrent_replays");
    // FP64 inner products on two streams
    const Geo &g0 = geos[0];
    double *d = (double *)dev_alloc(4 * sizeof(double));
    rc = radon_dot_f64(keep[0], keep[0], (int64_t)g0.nx, dt, d, A);
    const double ref = d[0];
    emu::begin_capture(A);
    rc |= radon_dot_f64(keep[0], keep[0], (int64_t)g0.nx, dt, d + 1, A);
    auto dot_a = emu::end_capture(A);
    emu::begin_capture(B);
    rc |= radon_dot_f64(keep[0], keep[0], (int64_t)g0.nx, dt, d + 2, B);
    auto dot_b = emu::end_capture(B);
    differ = false;
    for (size_t i = 0; i < dot_a.size() && i < dot_b.size(); ++i)
        differ = differ || dot_a[i].args != dot_b[i].args;
    expect(rc == 0 && !dot_a.empty() && dot_a.size() == dot_b.size() && differ,
           "dot_streams_use_own_partials");
    std::thread da([&] { emu::replay_graph(dot_a); });
    std::thread db([&] { emu::replay_graph(dot_b); });
    da.join();
    db.join();
    expect(d[1] == ref && d[2] == ref, "dot_concurrent_replays");
    // the no-allocation batched inner product: captured from its very first call,
    // bitwise equal to radon_dot_f64_batched, then a second, smaller call; a request
    // beyond its fixed scratch is rejected before anything is launched
    const int64_t m = (int64_t)g0.nx / 2;
    double *e = (double *)dev_alloc(8 * sizeof(double));
    hipStream_t C = reinterpret_cast<hipStream_t>(0x3000);
    emu::begin_capture(C);
    int rc_n = radon_dot_f64_batched_noalloc(keep[0], keep[0], m, 2, dt, e, C);
    auto dot_c = emu::end_capture(C);
    emu::replay_graph(dot_c);
    rc_n |= radon_dot_f64_batched(keep[0], keep[0], m, 2, dt, e + 2, A);
    rc_n |= radon_dot_f64_batched_noalloc(keep[0], keep[0], m / 3, 1, dt, e + 4, A);
    rc_n |= radon_dot_f64_batched(keep[0], keep[0], m / 3, 1, dt, e + 5, A);
    expect(rc_n == 0 && !dot_c.empty() && e[0] == e[2] && e[1] == e[3] && e[4] == e[5] &&
               e[0] > 0.0 && e[4] > 0.0,
           "noalloc_dot_equals_dot");
    expect(radon_dot_f64_batched_noalloc(keep[0], keep[0], 300000, 1025, dt, e, A) ==
               RADON_ERR_SCRATCH,
           "noalloc_dot_rejects_oversize");
    std::free(e);
    expect(emu::capture().allocs_while_capturing == 0, "no_allocation_under_capture");
    std::printf("summary geometries %zu failures %d\n", geos.size(), fails);
    std::free(d);
    for (void *p : outs) std::free(p);
    for (void *p : eager) std::free(p);
    for (void *p : keep) std::free(p);
    return fails ? 1 : 0;
}

// "shearlet" mode: argv[1] holds lines "W H batch dtype J alpha_0 .. alpha_{J-1}"; for
// each, random images x and random coefficients d (seeded), the forward transform of x
// and the adjoint of d through the emulated kernels; writes x, forward(x), d and
// adjoint(d) (FP64, storage-rounded inputs) to argv[3].
static int shearlet_mode(const char *spec, const char *path) {
    FILE *f = std::fopen(spec, "r");
    FILE *out = std::fopen(path, "wb");
    if (!f || !out) return 2;
    std::mt19937 rng(11);
    std::normal_distribution<float> normal;
    int fails = 0, W, H, B, dt, J;
    while (std::fscanf(f, "%d %d %d %d %d", &W, &H, &B, &dt, &J) == 5) {
        std::vector<double> alphas(J);
        for (double &a : alphas)
            if (std::fscanf(f, "%lf", &a) != 1) return 2;
        radon_shearlet_t sh{W, H, J, 0, alphas.data()};
        const int M = radon_shearlet_channels(&sh);
        if (M <= 0) return 2;
        const size_t es = esize(dt), nx = (size_t)B * W * H, nc = nx * M;
        void *x = dev_alloc(nx * es), *c = dev_alloc(nc * es), *d = dev_alloc(nc * es), *y = dev_alloc(nx * es);
        for (size_t i = 0; i < nx; ++i) from_float(x, i, normal(rng), dt);
        for (size_t i = 0; i < nc; ++i) from_float(d, i, normal(rng), dt);
        std::fprintf(stderr, "[emu] shearlet %dx%d batch %d dtype %d channels %d\n", W, H, B, dt, M);
        int rc = radon_shearlet_forward(&sh, x, c, B, dt, nullptr);
        if (!rc) rc = radon_shearlet_adjoint(&sh, d, y, B, dt, nullptr);
        if (rc) {
            std::printf("shearlet %dx%d status %d\n", W, H, rc);
            ++fails;
        }
        std::vector<double> buf(nc);
        auto dump = [&](const void *p, size_t n) {
            for (size_t i = 0; i < n; ++i) buf[i] = rc ? 0.0 : to_double(p, i, dt);
            std::fwrite(buf.data(), sizeof(double), n, out);
        };
        dump(x, nx);
        dump(c, nc);
        dump(d, nc);
        dump(y, nx);
        std::free(x);
        std::free(c);
        std::free(d);
        std::free(y);
    }
    std::fclose(f);
    std::fclose(out);
    std::printf("summary shearlet failures %d\n", fails);
    return fails ? 1 : 0;
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    if (argc > 3 && std::strcmp(argv[2], "shearlet") == 0) return shearlet_mode(argv[1], argv[3]);
    const bool batched = argc > 2 && std::strcmp(argv[2], "batched") == 0;
    const bool filtering = argc > 3 && std::strcmp(argv[2], "filter") == 0;
    const bool solving = argc > 5 && std::strcmp(argv[2], "solver") == 0;
    const bool lifetime = argc > 2 && std::strcmp(argv[2], "lifetime") == 0;
    FILE *f = std::fopen(argv[1], "r");
    if (!f) return 2;
    std::vector<Geo> geos;
    for (;;) {
        Geo g;
        if (std::fscanf(f, "%d %d %d %lf %lf %lf %lf %d %d %d", &g.beam, &g.n, &g.D, &g.sp, &g.S,
                        &g.E, &g.step, &g.batch, &g.dt, &g.A) != 10)
            break;
        g.angles.resize(g.A);
        for (double &a : g.angles)
            if (std::fscanf(f, "%lf", &a) != 1) return 2;
        geos.push_back(std::move(g));
    }
    std::fclose(f);
    std::mt19937 rng(7);
    std::normal_distribution<float> normal;
    int fails = 0;
    for (size_t k = 0; k < geos.size(); ++k) {
        Geo &g = geos[k];
        if (solving || lifetime) {
            g.g = radon_geometry_t{g.beam, g.n, g.A, g.D, g.angles.data(), g.sp, g.S, g.E, g.step};
            g.nx = (size_t)g.batch * g.n * g.n;
            g.ny = (size_t)g.batch * g.A * g.D;
            g.x.resize(g.nx * esize(g.dt));
            g.y.resize(g.ny * esize(g.dt));
            for (size_t i = 0; i < g.nx; ++i) from_float(g.x.data(), i, normal(rng), g.dt);
            for (size_t i = 0; i < g.ny; ++i) from_float(g.y.data(), i, normal(rng), g.dt);
            continue;
        }
        if (filtering) {
            g.g = radon_geometry_t{g.beam, g.n, g.A, g.D, g.angles.data(), g.sp, g.S, g.E, g.step};
            g.nx = (size_t)g.batch * g.n * g.n;
            g.ny = (size_t)g.batch * g.A * g.D;
            g.y.resize(g.ny * esize(g.dt));
            for (size_t i = 0; i < g.ny; ++i) from_float(g.y.data(), i, normal(rng), g.dt);
            continue;
        }
        g.g = radon_geometry_t{g.beam, g.n, g.A, g.D, g.angles.data(), g.sp, g.S, g.E, g.step};
        g.nx = (size_t)g.batch * g.n * g.n;
        g.ny = (size_t)g.batch * g.A * g.D;
        const size_t es = esize(g.dt);
        g.x.resize(g.nx * es);
        g.y.resize(g.ny * es);
        for (size_t i = 0; i < g.nx; ++i) from_float(g.x.data(), i, normal(rng), g.dt);
        for (size_t i = 0; i < g.ny; ++i) from_float(g.y.data(), i, normal(rng), g.dt);
        std::fprintf(stderr, "[emu] geometry %zu: beam %d N %d A %d D %d batch %d dtype %d\n", k,
                     g.beam, g.n, g.A, g.D, g.batch, g.dt);
        void *xin = dev_alloc(g.nx * es), *yin = dev_alloc(g.ny * es);
        std::memcpy(xin, g.x.data(), g.nx * es);
        std::memcpy(yin, g.y.data(), g.ny * es);
        g.fx = dev_alloc(g.ny * es);
        g.bx = dev_alloc(g.nx * es);
        void *fd = dev_alloc(g.ny * es), *bd = dev_alloc(g.nx * es);
        int rc = radon_forward(&g.g, xin, g.fx, g.batch, g.dt, 1.0f, nullptr);
        if (!rc) rc = radon_backproject(&g.g, yin, g.bx, g.batch, g.dt, 1.0f, nullptr);
        int info[10] = {0};
        if (!rc) rc = radon_plan_info(&g.g, g.dt, g.batch, info);
        // direct kernels: plans rebuilt with the tiled planners switched off
        if (!rc) {
            radon_release_plans();
            setenv("RADON_VARIANT", "direct", 1);
            rc = radon_forward(&g.g, xin, fd, g.batch, g.dt, 1.0f, nullptr);
            if (!rc) rc = radon_backproject(&g.g, yin, bd, g.batch, g.dt, 1.0f, nullptr);
            unsetenv("RADON_VARIANT");
            radon_release_plans();
        }
        if (rc) {
            std::printf("geometry %zu status %d\n", k, rc);
            ++fails;
            continue;
        }
        // oracle on the same (already rounded) inputs
        std::vector<double> xd(g.nx), yd(g.ny), of(g.ny), ob(g.nx);
        for (size_t i = 0; i < g.nx; ++i) xd[i] = to_double(g.x.data(), i, g.dt);
        for (size_t i = 0; i < g.ny; ++i) yd[i] = to_double(g.y.data(), i, g.dt);
        oracle_forward(g.beam, g.n, g.A, g.angles.data(), g.D, g.sp, g.S, g.E, g.step, xd.data(),
                       g.batch, 1.0, of.data());
        oracle_backproject(g.beam, g.n, g.A, g.angles.data(), g.D, g.sp, g.S, g.E, g.step,
                           yd.data(), g.batch, 1.0, ob.data());
        const double ef = rel_l2(g.fx, g.dt, of.data(), g.ny), eb = rel_l2(g.bx, g.dt, ob.data(), g.nx);
        g.oracle_fx = of;
        const double df = rel_l2(fd, g.dt, of.data(), g.ny), db = rel_l2(bd, g.dt, ob.data(), g.nx);
        std::printf("geometry %zu fwd_variant %d bp_variant %d forward %.3e backprojection %.3e "
                    "direct_forward %.3e direct_backprojection %.3e\n",
                    k, info[3], info[8], ef, eb, df, db);
        std::free(xin);
        std::free(yin);
        std::free(fd);
        std::free(bd);
    }
    if (filtering) return filter_mode(geos, argv[3]);
    if (lifetime) return geos.empty() ? 2 : lifetime_mode(geos);
    if (solving) {
        char *end = nullptr;
        const double alpha = std::strtod(argv[4], &end);
        if (end == argv[4] || *end) return 2;     // the step must be a plain number
        return solver_mode(geos, argv[3], alpha, std::atoi(argv[5]));
    }
    if (batched) {
        std::vector<radon_job_t> jf, jb;
        std::vector<void *> of, ob, ins;
        for (Geo &g : geos) {
            const size_t es = esize(g.dt);
            void *xin = dev_alloc(g.nx * es), *yin = dev_alloc(g.ny * es);
            std::memcpy(xin, g.x.data(), g.nx * es);
            std::memcpy(yin, g.y.data(), g.ny * es);
            of.push_back(dev_alloc(g.ny * es));
            ob.push_back(dev_alloc(g.nx * es));
            ins.push_back(xin);
            ins.push_back(yin);
            jf.push_back(radon_job_t{&g.g, xin, of.back(), g.batch, 1.0f});
            jb.push_back(radon_job_t{&g.g, yin, ob.back(), g.batch, 1.0f});
        }
        const int dt = geos.empty() ? RADON_F32 : geos[0].dt;
        std::fprintf(stderr, "[emu] batched forward and backprojection of %zu jobs\n", geos.size());
        int rc = radon_forward_batched(jf.data(), (int)jf.size(), dt, nullptr);
        if (!rc) rc = radon_backproject_batched(jb.data(), (int)jb.size(), dt, nullptr);
        // FP32: bitwise equal to the per-call results.  16-bit: the batched forward takes
        // tap pairs along x (weights rounded to the storage type), so it is held to the
        // 16-bit bar against the oracle instead; the backprojection is bitwise.
        int same = 0;
        for (size_t k = 0; !rc && k < geos.size(); ++k) {
            const Geo &g = geos[k];
            const size_t es = esize(g.dt);
            bool fwd_ok;
            if (g.dt == RADON_F32) {
                fwd_ok = std::memcmp(of[k], g.fx, g.ny * es) == 0;
            } else {
                const double e = g.oracle_fx.size() == g.ny ? rel_l2(of[k], g.dt, g.oracle_fx.data(), g.ny) : 1.0;
                std::printf("batched 16-bit forward %zu: rel L2 to the oracle %.3e\n", k, e);
                fwd_ok = e <= 5e-3;
            }
            same += fwd_ok && std::memcmp(ob[k], g.bx, g.nx * es) == 0;
        }
        std::printf("batched status %d identical %d of %zu\n", rc, same, geos.size());
        if (rc || same != (int)geos.size()) ++fails;
    }
    std::printf("summary geometries %zu failures %d\n", geos.size(), fails);
    return fails ? 1 : 0;
}
