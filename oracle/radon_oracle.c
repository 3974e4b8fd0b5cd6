/*
 * Oracle for the discretised Radon transform: a plain, slow FP64 CPU
 * implementation used ONLY as test infrastructure (pytest, the smoke check and
 * the benchmark's CPU-baseline leg).  The product path never calls it.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * What is computed.  The paper (TorchRadon, arXiv 2009.14788) gives the API and
 * the geometry in words only: parallel beam (Sec. 3.1.1), flat-detector fan
 * beam with a point source at `source_distance` and a detector line at
 * `det_distance` from the centre (Sec. 3.1.2), forward projection and the
 * backprojection used as its adjoint inside CG (Sec. 4.3), batch processing
 * (Sec. 4.1).  The discrete operator is the ray-driven one: each line integral
 * is sampled along the ray with bilinear interpolation and multiplied by the
 * step length; the backprojection is the exact transpose.  The readings taken
 * where the paper is silent (pixel centres, angle convention, bin centres,
 * foot-point sample lattice, zero padding) are:
 *
 *   image x[r][c], 0 <= r,c < N, pixel centre (X_c, Y_r) = (c-(N-1)/2, r-(N-1)/2)
 *   tent  L(t) = max(0, 1-|t|);  f(P) = sum_{r,c} x[r][c] L(P_x-X_c) L(P_y-Y_r)
 *   angle th: detector axis u = (cos th, sin th), ray axis v = (-sin th, cos th)
 *   bin d: s_d = (d-(D-1)/2) * spacing
 *   ray (th, d): the line through the foot point F (the point of the ray
 *     closest to the rotation centre) with unit direction w
 *       parallel: F = s_d u, w = v
 *       fan:      source at -S v, detector point at E v + s_d u,
 *                 w = unit vector from source to detector point,
 *                 F = orthogonal projection of the origin onto the ray
 *   samples P_k = F + k*dt*w for every integer k
 *   forward       y[a][d] = scale * dt * sum_k f(P_k)
 *   backprojection         = scale * (transpose of the same matrix)
 *
 * Every sum over k runs over a range that contains every sample inside the
 * open support box |P_x|,|P_y| < (N+1)/2; samples outside contribute exactly 0.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int beam;               /* 0 = parallel, 1 = flat-detector fan */
    int n;                  /* image side N */
    int n_angles;           /* A */
    const double *angles;   /* [A] radians */
    int det_count;          /* D */
    double det_spacing;     /* detector bin spacing */
    double source_distance; /* S, fan only */
    double det_distance;    /* E, fan only */
    double step;            /* dt, sample spacing along the ray */
} oracle_geom;

typedef struct { double fx, fy, wx, wy; } oracle_ray;

static double tent(double t)
{
    double a = 1.0 - fabs(t);
    return a > 0.0 ? a : 0.0;
}

/* Ray (angle index a, bin d) as foot point + unit direction (Sec. 3.1.1 and
 * 3.1.2 geometry, with the conventions listed in the file header). */
static oracle_ray ray_of(const oracle_geom *g, int a, int d)
{
    double th = g->angles[a];
    double ux = cos(th), uy = sin(th);
    double vx = -uy, vy = ux;
    double s = ((double)d - 0.5 * (double)(g->det_count - 1)) * g->det_spacing;
    oracle_ray r;
    if (g->beam == 0) {
        r.fx = s * ux;
        r.fy = s * uy;
        r.wx = vx;
        r.wy = vy;
    } else {
        double S = g->source_distance, E = g->det_distance;
        double srcx = -S * vx, srcy = -S * vy;            /* point source */
        double detx = E * vx + s * ux, dety = E * vy + s * uy; /* bin centre */
        double dx = detx - srcx, dy = dety - srcy;
        double len = sqrt(dx * dx + dy * dy);
        r.wx = dx / len;
        r.wy = dy / len;
        /* foot point: source minus its component along w */
        double along = srcx * r.wx + srcy * r.wy;
        r.fx = srcx - along * r.wx;
        r.fy = srcy - along * r.wy;
    }
    return r;
}

/* Bilinear interpolant of one image with zero outside, at centred point P. */
static double bilinear(const double *img, int n, double px, double py)
{
    double h = 0.5 * (double)(n - 1);
    double cx = px + h, cy = py + h;   /* fractional column / row index */
    int c0 = (int)floor(cx), r0 = (int)floor(cy);
    double v = 0.0;
    for (int r = r0; r <= r0 + 1; ++r) {
        if (r < 0 || r >= n) continue;
        double wy = tent(cy - (double)r);
        for (int c = c0; c <= c0 + 1; ++c) {
            if (c < 0 || c >= n) continue;
            v += img[(size_t)r * n + c] * tent(cx - (double)c) * wy;
        }
    }
    return v;
}

/* Integer range [*klo, *khi] holding every sample of the ray inside the open
 * support box, widened by one on each side (the extra samples add 0). */
static void k_range(const oracle_geom *g, const oracle_ray *ry, long *klo, long *khi)
{
    double b = 0.5 * (double)(g->n + 1);
    double tlo = -INFINITY, thi = INFINITY;
    double f[2] = {ry->fx, ry->fy}, w[2] = {ry->wx, ry->wy};
    for (int i = 0; i < 2; ++i) {
        if (w[i] != 0.0) {
            double t1 = (-b - f[i]) / w[i], t2 = (b - f[i]) / w[i];
            if (t1 > t2) { double t = t1; t1 = t2; t2 = t; }
            if (t1 > tlo) tlo = t1;
            if (t2 < thi) thi = t2;
        } else if (fabs(f[i]) >= b) {
            tlo = 1.0; thi = -1.0;   /* the ray misses the box */
        }
    }
    if (!(tlo <= thi)) { *klo = 0; *khi = -1; return; }
    *klo = (long)floor(tlo / g->step) - 1;
    *khi = (long)ceil(thi / g->step) + 1;
}

static int check_geom(const oracle_geom *g)
{
    if (g->n <= 0 || g->n_angles <= 0 || g->det_count <= 0) return -1;
    if (!(g->det_spacing > 0.0) || !(g->step > 0.0)) return -1;
    if (g->beam != 0 && g->beam != 1) return -1;
    if (g->beam == 1 && (!(g->source_distance > 0.0) || !(g->det_distance >= 0.0))) return -1;
    return 0;
}

#define GEOM_ARGS int beam, int n, int n_angles, const double *angles, int det_count, \
    double det_spacing, double source_distance, double det_distance, double step
#define MAKE_GEOM oracle_geom g = {beam, n, n_angles, angles, det_count, det_spacing, \
    source_distance, det_distance, step}

/* Forward projection of B images x[B][N][N] into y[B][A][D]. */
int oracle_forward(GEOM_ARGS, const double *x, int batch, double scale, double *y)
{
    MAKE_GEOM;
    if (check_geom(&g)) return -1;
    long total = (long)batch * g.n_angles;
#pragma omp parallel for schedule(dynamic, 1)
    for (long ba = 0; ba < total; ++ba) {
        long b = ba / g.n_angles;
        int a = (int)(ba % g.n_angles);
        const double *img = x + (size_t)b * g.n * g.n;
        for (int d = 0; d < g.det_count; ++d) {
            oracle_ray ry = ray_of(&g, a, d);
            long klo, khi;
            k_range(&g, &ry, &klo, &khi);
            double acc = 0.0;
            for (long k = klo; k <= khi; ++k) {
                double t = (double)k * g.step;
                acc += bilinear(img, g.n, ry.fx + t * ry.wx, ry.fy + t * ry.wy);
            }
            y[((size_t)b * g.n_angles + a) * g.det_count + d] = scale * g.step * acc;
        }
    }
    return 0;
}

/* Scatter of the rays of angles [a0, a1) of one sinogram into acc[N][N]: every
 * sample of every ray hands its value, times its four bilinear weights, to the
 * pixels it was interpolated from. */
static void scatter_angles(const oracle_geom *g, const double *sino, double scale, int a0,
                           int a1, double *acc)
{
    double h = 0.5 * (double)(g->n - 1);
    for (int a = a0; a < a1; ++a) {
        for (int d = 0; d < g->det_count; ++d) {
            double val = scale * g->step * sino[(size_t)a * g->det_count + d];
            oracle_ray ry = ray_of(g, a, d);
            long klo, khi;
            k_range(g, &ry, &klo, &khi);
            for (long k = klo; k <= khi; ++k) {
                double t = (double)k * g->step;
                double cx = ry.fx + t * ry.wx + h, cy = ry.fy + t * ry.wy + h;
                int c0 = (int)floor(cx), r0 = (int)floor(cy);
                for (int r = r0; r <= r0 + 1; ++r) {
                    if (r < 0 || r >= g->n) continue;
                    double wy = tent(cy - (double)r);
                    for (int c = c0; c <= c0 + 1; ++c) {
                        if (c < 0 || c >= g->n) continue;
                        acc[(size_t)r * g->n + c] += val * tent(cx - (double)c) * wy;
                    }
                }
            }
        }
    }
}

/* Backprojection y[B][A][D] -> x[B][N][N] in scatter form, the literal transpose
 * of oracle_forward.  The angles of each image are cut into a fixed number of
 * contiguous blocks (independent of the thread count); every block scatters into
 * its own accumulator and the accumulators are added in block order, so the
 * result is the same on any number of threads.  Returns -2 if the accumulators
 * cannot be allocated. */
int oracle_backproject(GEOM_ARGS, const double *y, int batch, double scale, double *x)
{
    MAKE_GEOM;
    if (check_geom(&g)) return -1;
    const size_t npix = (size_t)g.n * g.n;
    int nblk = g.n_angles < 32 ? g.n_angles : 32;
    const size_t cap = ((size_t)512 << 20) / (npix * sizeof(double));
    if ((size_t)nblk > cap) nblk = cap > 0 ? (int)cap : 1;
    double *part = (double *)malloc((size_t)nblk * npix * sizeof(double));
    if (!part) return -2;
    for (long b = 0; b < batch; ++b) {
        const double *sino = y + (size_t)b * g.n_angles * g.det_count;
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k < nblk; ++k) {
            double *acc = part + (size_t)k * npix;
            memset(acc, 0, npix * sizeof(double));
            scatter_angles(&g, sino, scale, (int)((long)k * g.n_angles / nblk),
                           (int)((long)(k + 1) * g.n_angles / nblk), acc);
        }
        double *img = x + (size_t)b * npix;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < (long)npix; ++i) {
            double v = 0.0;
            for (int k = 0; k < nblk; ++k) v += part[(size_t)k * npix + i];
            img[i] = v;
        }
    }
    free(part);
    return 0;
}

/* One system-matrix entry R[(a,d),(r,c)] = dt * sum_k L(P_kx-X_c) L(P_ky-Y_r),
 * with k over a window around the pixel: only samples within distance sqrt(2)
 * of the pixel centre can have both tents non-zero. */
double oracle_matrix_entry(GEOM_ARGS, int a, int d, int r, int c)
{
    MAKE_GEOM;
    if (check_geom(&g)) return NAN;
    oracle_ray ry = ray_of(&g, a, d);
    double h = 0.5 * (double)(g.n - 1);
    double qx = (double)c - h, qy = (double)r - h;
    double tc = (qx - ry.fx) * ry.wx + (qy - ry.fy) * ry.wy; /* pixel centre along the ray */
    long klo = (long)floor((tc - 1.5) / g.step) - 1;
    long khi = (long)ceil((tc + 1.5) / g.step) + 1;
    double acc = 0.0;
    for (long k = klo; k <= khi; ++k) {
        double t = (double)k * g.step;
        double px = ry.fx + t * ry.wx, py = ry.fy + t * ry.wy;
        acc += tent(px - qx) * tent(py - qy);
    }
    return g.step * acc;
}

/* Dense system matrix R[A*D][N*N] (row = ray a*D+d, column = pixel r*N+c),
 * entry by entry.  Only for small N. */
int oracle_dense_matrix(GEOM_ARGS, double *mat)
{
    MAKE_GEOM;
    if (check_geom(&g)) return -1;
    long rows = (long)g.n_angles * g.det_count, cols = (long)g.n * g.n;
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < rows; ++i) {
        int a = (int)(i / g.det_count), d = (int)(i % g.det_count);
        for (long j = 0; j < cols; ++j)
            mat[i * cols + j] = oracle_matrix_entry(beam, n, n_angles, angles, det_count,
                det_spacing, source_distance, det_distance, step, a, d, (int)(j / g.n), (int)(j % g.n));
    }
    return 0;
}

/* Selected forward outputs y[b][a][d] for idx = n triples (b, a, d). */
int oracle_forward_rays(GEOM_ARGS, const double *x, double scale, long n_idx,
                        const int64_t *idx, double *out)
{
    MAKE_GEOM;
    if (check_geom(&g)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n_idx; ++i) {
        long b = (long)idx[3 * i];
        int a = (int)idx[3 * i + 1], d = (int)idx[3 * i + 2];
        const double *img = x + (size_t)b * g.n * g.n;
        oracle_ray ry = ray_of(&g, a, d);
        long klo, khi;
        k_range(&g, &ry, &klo, &khi);
        double acc = 0.0;
        for (long k = klo; k <= khi; ++k) {
            double t = (double)k * g.step;
            acc += bilinear(img, g.n, ry.fx + t * ry.wx, ry.fy + t * ry.wy);
        }
        out[i] = scale * g.step * acc;
    }
    return 0;
}

/* Selected backprojection outputs x[b][r][c] for idx = n triples (b, r, c),
 * each as the column sum  scale * sum_{a,d} y[b][a][d] R[(a,d),(r,c)]. */
int oracle_backproject_pixels(GEOM_ARGS, const double *y, double scale, long n_idx,
                              const int64_t *idx, double *out)
{
    MAKE_GEOM;
    if (check_geom(&g)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n_idx; ++i) {
        long b = (long)idx[3 * i];
        int r = (int)idx[3 * i + 1], c = (int)idx[3 * i + 2];
        double acc = 0.0;
        for (int a = 0; a < g.n_angles; ++a) {
            const double *row = y + ((size_t)b * g.n_angles + a) * g.det_count;
            for (int d = 0; d < g.det_count; ++d) {
                if (row[d] == 0.0) continue;
                acc += row[d] * oracle_matrix_entry(beam, n, n_angles, angles, det_count,
                    det_spacing, source_distance, det_distance, step, a, d, r, c);
            }
        }
        out[i] = scale * acc;
    }
    return 0;
}

/* Threads the OpenMP loops use from now on (n >= 1); for timing only. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
