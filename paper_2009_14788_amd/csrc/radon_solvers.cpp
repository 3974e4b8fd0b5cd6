// Landweber iteration and conjugate gradient on the normal equations (TorchRadon
// Sec. 4.2) as loops of launches queued on one stream: the projections are the
// library's own forward and backprojection, the inner products and updates the
// per-system vector kernels.  No step waits on the host: every CG coefficient is a
// ratio of FP64 inner products that the update kernel reads from device memory.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "../../include/radon.h"
#include "radon_common.hpp"
#include "radon_launch.hpp"

namespace {

using namespace radon;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Byte offsets of the solver buffers inside the caller's workspace.
struct SolverLayout {
    size_t r = 0, q = 0, s = 0, p = 0, ss0 = 0, ss1 = 0, qq = 0, partials = 0, total = 0;
};

SolverLayout layout(const radon_geometry_t *g, int solver, int batch, int dtype) {
    const size_t es = dtype == RADON_F32 ? 4 : 2;
    const size_t ny = align256((size_t)batch * g->n_angles * g->det_count * es);
    const size_t nx = align256((size_t)batch * g->image_size * g->image_size * es);
    const size_t nd = align256((size_t)batch * sizeof(double));
    SolverLayout L;
    L.r = 0;
    if (solver == RADON_SOLVER_LANDWEBER) {
        L.s = ny;                        // the scaled gradient alpha R^T (R x - y)
        L.total = ny + nx;
        return L;
    }
    L.q = ny;
    L.s = 2 * ny;
    L.p = 2 * ny + nx;
    L.ss0 = 2 * ny + 2 * nx;
    L.ss1 = L.ss0 + nd;
    L.qq = L.ss1 + nd;
    L.partials = L.qq + nd;
    L.total = L.partials + align256((size_t)batch * kDotRowChunks * sizeof(double));
    return L;
}

int check_args(const radon_geometry_t *g, const void *y, void *x, int32_t batch, int32_t iterations,
               int32_t dtype, void *ws, int64_t ws_bytes, int solver) {
    int rc = radon_validate(g);
    if (rc != RADON_OK) return rc;
    if (dtype != RADON_F32 && dtype != RADON_F16 && dtype != RADON_BF16) return RADON_ERR_INVALID_ARG;
    if (batch < 0 || batch > 65535 || iterations < 0 || ws_bytes < 0) return RADON_ERR_INVALID_ARG;
    if (batch == 0 || iterations == 0) return RADON_OK;
    for (const void *p : {(const void *)y, (const void *)x, (const void *)ws}) {
        if (!p) return RADON_ERR_INVALID_ARG;
        if (reinterpret_cast<uintptr_t>(p) & 15u) return RADON_ERR_ALIGN;
    }
    if ((size_t)ws_bytes < layout(g, solver, batch, dtype).total) return RADON_ERR_INVALID_ARG;
    return RADON_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? RADON_OK : RADON_ERR_HIP; }

}  // namespace

extern "C" {

int64_t radon_solver_workspace_bytes(const radon_geometry_t *geometry, int32_t solver,
                                     int32_t batch, int32_t dtype) {
    int rc = radon_validate(geometry);
    if (rc != RADON_OK) return rc;
    if (solver != RADON_SOLVER_LANDWEBER && solver != RADON_SOLVER_CGNE) return RADON_ERR_INVALID_ARG;
    if (dtype != RADON_F32 && dtype != RADON_F16 && dtype != RADON_BF16) return RADON_ERR_INVALID_ARG;
    if (batch < 0 || batch > 65535) return RADON_ERR_INVALID_ARG;
    return (int64_t)layout(geometry, solver, batch, dtype).total;
}

int radon_landweber(const radon_geometry_t *geometry, const void *y, void *x, int32_t batch,
                    double alpha, int32_t iterations, int32_t dtype, void *workspace,
                    int64_t workspace_bytes, void *stream) {
    if (!std::isfinite(alpha) || !std::isfinite((float)alpha)) return RADON_ERR_INVALID_ARG;
    int rc = check_args(geometry, y, x, batch, iterations, dtype, workspace, workspace_bytes,
                        RADON_SOLVER_LANDWEBER);
    if (rc != RADON_OK || batch == 0 || iterations == 0) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SolverLayout L = layout(geometry, RADON_SOLVER_LANDWEBER, batch, dtype);
    char *ws = static_cast<char *>(workspace);
    void *r = ws + L.r, *grad = ws + L.s;
    const long long nx = (long long)geometry->image_size * geometry->image_size;
    const long long ny = (long long)geometry->n_angles * geometry->det_count;
    for (int k = 0; k < iterations; ++k) {
        if ((rc = radon_forward(geometry, x, r, batch, dtype, 1.0f, stream)) != RADON_OK) return rc;
        if ((rc = hip_status(launch_axpy_ratio(r, y, r, nullptr, nullptr, -1.0, ny, batch, dtype, s))))
            return rc;
        if ((rc = radon_backproject(geometry, r, grad, batch, dtype, (float)alpha, stream)) != RADON_OK)
            return rc;
        if ((rc = hip_status(launch_axpy_ratio(x, grad, x, nullptr, nullptr, -1.0, nx, batch, dtype, s))))
            return rc;
    }
    return RADON_OK;
}

int radon_cgne(const radon_geometry_t *geometry, const void *y, void *x, int32_t batch,
               int32_t iterations, int32_t dtype, void *workspace, int64_t workspace_bytes,
               void *stream) {
    int rc = check_args(geometry, y, x, batch, iterations, dtype, workspace, workspace_bytes,
                        RADON_SOLVER_CGNE);
    if (rc != RADON_OK) return rc;
    if (dtype != RADON_F32) return RADON_ERR_UNSUPPORTED;
    if (batch == 0 || iterations == 0) return RADON_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SolverLayout L = layout(geometry, RADON_SOLVER_CGNE, batch, dtype);
    char *ws = static_cast<char *>(workspace);
    void *r = ws + L.r, *q = ws + L.q, *sv = ws + L.s, *p = ws + L.p;
    double *ss[2] = {reinterpret_cast<double *>(ws + L.ss0), reinterpret_cast<double *>(ws + L.ss1)};
    double *qq = reinterpret_cast<double *>(ws + L.qq);
    double *partials = reinterpret_cast<double *>(ws + L.partials);
    const long long nx = (long long)geometry->image_size * geometry->image_size;
    const long long ny = (long long)geometry->n_angles * geometry->det_count;
    // r = y - R x;  s = R^T r;  p = s;  ss = <s, s>
    if ((rc = radon_forward(geometry, x, r, batch, dtype, 1.0f, stream)) != RADON_OK) return rc;
    if ((rc = hip_status(launch_axpy_ratio(y, r, r, nullptr, nullptr, -1.0, ny, batch, dtype, s))))
        return rc;
    if ((rc = radon_backproject(geometry, r, sv, batch, dtype, 1.0f, stream)) != RADON_OK) return rc;
    if ((rc = hip_status(launch_axpy_ratio(sv, sv, p, nullptr, nullptr, 0.0, nx, batch, dtype, s))))
        return rc;
    if ((rc = hip_status(launch_dot_rows(sv, sv, nx, batch, dtype, ss[0], partials, s)))) return rc;
    for (int k = 0; k < iterations; ++k) {
        double *cur = ss[k & 1], *nxt = ss[(k + 1) & 1];
        // q = R p;  a = <s,s> / <q,q>;  x += a p;  r -= a q
        if ((rc = radon_forward(geometry, p, q, batch, dtype, 1.0f, stream)) != RADON_OK) return rc;
        if ((rc = hip_status(launch_dot_rows(q, q, ny, batch, dtype, qq, partials, s)))) return rc;
        if ((rc = hip_status(launch_axpy_ratio(x, p, x, cur, qq, 1.0, nx, batch, dtype, s)))) return rc;
        if ((rc = hip_status(launch_axpy_ratio(r, q, r, cur, qq, -1.0, ny, batch, dtype, s)))) return rc;
        // s' = R^T r;  p = s' + (<s',s'> / <s,s>) p
        if ((rc = radon_backproject(geometry, r, sv, batch, dtype, 1.0f, stream)) != RADON_OK) return rc;
        if ((rc = hip_status(launch_dot_rows(sv, sv, nx, batch, dtype, nxt, partials, s)))) return rc;
        if ((rc = hip_status(launch_axpy_ratio(sv, p, p, nxt, cur, 1.0, nx, batch, dtype, s)))) return rc;
    }
    return RADON_OK;
}

}  // extern "C"
