/*
 * radon.h -- C ABI of libradon.so, the MI355X (gfx950) discretised Radon transform.
 *
 * The operator (TorchRadon, arXiv 2009.14788; geometry of Sec. 3.1.1 and 3.1.2,
 * batch processing of Sec. 4.1, 16-bit storage with 32-bit arithmetic of Sec. 3.3,
 * backprojection used as the adjoint of the projection in Sec. 4.3):
 *
 *   image x[r][c], 0 <= r,c < N, pixel centre (c-(N-1)/2, r-(N-1)/2), pixel size 1;
 *   f = bilinear interpolant of x with zeros outside the image;
 *   angle t: detector axis u = (cos t, sin t), ray axis v = (-sin t, cos t);
 *   bin d: s_d = (d-(D-1)/2) * det_spacing;
 *   parallel beam: ray through s_d*u along v;
 *   fan beam: point source at -S*v, flat detector through E*v along u, the ray
 *     joins the source and the bin centre E*v + s_d*u;
 *   each ray is sampled at P_k = F + k*step*w (F = the ray's point closest to the
 *     rotation centre, w = its unit direction, k any integer);
 *   forward         y[a][d] = scale * step * sum_k f(P_k)            (y = scale*R x)
 *   backprojection  x       = scale * R^T y (the exact transpose, no other factor).
 *
 * Layouts.  Images: x[B][N][N] contiguous, row-major.  Sinograms: y[B][A][D]
 * contiguous.  Element type per call: RADON_F32, RADON_F16 or RADON_BF16; 16-bit
 * values are widened exactly to FP32, all arithmetic and accumulation is FP32, and
 * each output is rounded once (round-to-nearest-even) on store; FP16 overflow
 * stores +-inf.
 *
 * Ownership.  The caller owns every data buffer (device memory); the library never
 * frees, keeps or reallocates them.  Calls are asynchronous on `stream` (a
 * hipStream_t passed as void*, NULL = the null stream); buffers must stay alive
 * until the stream's work has completed.  The library owns only its per-geometry
 * plans (angle/ray tables, work items, launch shapes), one workspace per (device,
 * stream) for the interleaved copy of a call's input (grown on demand, never under
 * stream capture), the tables of uneven batches with one work counter per stream,
 * and the inner products' partial sums per (device, stream); all are created on
 * first use (or by radon_prepare()) and kept until radon_release_plans().  A buffer
 * that a captured graph may still use (a replaced workspace or partials buffer, or
 * a batch table that a graph captured) is never freed before radon_release_plans().
 *
 * Errors.  Every entry point returns RADON_OK (0) or a negative status; no C++
 * exception crosses the ABI.  A launch error is reported from the call; a fault
 * during execution surfaces at the caller's next synchronisation.  batch == 0 is a
 * no-op returning RADON_OK.  Device pointers must be 16-byte aligned
 * (RADON_ERR_ALIGN).  Plans are built outside stream capture: a call on a capturing
 * stream whose plan does not exist yet returns RADON_ERR_NOT_PREPARED.
 */
#ifndef RADON_H
#define RADON_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RADON_OK = 0,
    RADON_ERR_INVALID_ARG = -1,   /* bad geometry, size, dtype or null pointer */
    RADON_ERR_ALIGN = -2,         /* a device pointer is not 16-byte aligned */
    RADON_ERR_UNSUPPORTED = -3,   /* valid request the library does not implement */
    RADON_ERR_HIP = -4,           /* a HIP runtime call or kernel launch failed */
    RADON_ERR_ALLOC = -5,         /* device or host allocation failed */
    RADON_ERR_NO_DEVICE = -6,     /* no usable GPU */
    RADON_ERR_NOT_PREPARED = -7,  /* plan missing while the stream is capturing */
    RADON_ERR_SCRATCH = -8        /* request exceeds a no-allocation entry point's fixed scratch */
};

enum { RADON_PARALLEL = 0, RADON_FANBEAM = 1 };
enum { RADON_F32 = 0, RADON_F16 = 1, RADON_BF16 = 2 };

/* Acquisition geometry (Sec. 3.1.1 parallel beam: image size, angles, detector count
 * and spacing; Sec. 3.1.2 fan beam: plus source and detector distances). */
typedef struct radon_geometry {
    int32_t beam;              /* RADON_PARALLEL or RADON_FANBEAM */
    int32_t image_size;        /* N >= 1 */
    int32_t n_angles;          /* A >= 1 */
    int32_t det_count;         /* D >= 1 */
    const double *angles;      /* host array [A] of angles in radians; read during the call */
    double det_spacing;        /* > 0 */
    double source_distance;    /* fan only: S > (N+1)/2*sqrt(2), source outside the image */
    double det_distance;       /* fan only: E >= 0 */
    double step;               /* sample spacing along each ray, > 0 (usual value 1) */
} radon_geometry_t;

/* Library utility (no operation of the paper): host-only check of a geometry against
 * the limits above (no device needed).  RADON_OK, RADON_ERR_INVALID_ARG, or
 * RADON_ERR_UNSUPPORTED for sizes past the kernels' index ranges; never touches the
 * GPU. */
int radon_validate(const radon_geometry_t *geometry);

/* Library utility (no operation of the paper; it prepares the batch processing of
 * Sec. 4.1): build (or find) the plan of a geometry on the current device for `dtype`
 * and a batch size: angle and ray tables, work items, the null stream's workspace, and
 * launch shapes chosen by timing the candidates on the device (unless the environment
 * sets RADON_AUTOTUNE=0; the choice is kept per storage type and power-of-two batch
 * class, in memory and, if RADON_TUNE_CACHE names a file, one text line per choice in
 * that file).  Synchronises the device.  Call before capturing a stream that will use
 * the geometry. */
int radon_prepare(const radon_geometry_t *geometry, int32_t dtype, int32_t batch);

/* Forward projection (Sec. 3.1, Sec. 4.1): y[b] = scale * R x[b] for b < batch.
 * x: device [batch][N][N], y: device [batch][A][D], both of `dtype`. */
int radon_forward(const radon_geometry_t *geometry, const void *x, void *y, int32_t batch,
                  int32_t dtype, float scale, void *stream);

/* Backprojection, the exact transpose of radon_forward (used as the adjoint in
 * Sec. 4.3): x[b] = scale * R^T y[b].  y: device [batch][A][D], x: device
 * [batch][N][N], both of `dtype`.  A gather over the rays through each pixel: no
 * atomics, deterministic. */
int radon_backproject(const radon_geometry_t *geometry, const void *y, void *x,
                      int32_t batch, int32_t dtype, float scale, void *stream);

/* One job of an uneven batch: `batch` images of one geometry. */
typedef struct radon_job {
    const radon_geometry_t *geometry;
    const void *input;     /* device: images (forward) or sinograms (backprojection) */
    void *output;          /* device: sinograms (forward) or images (backprojection) */
    int32_t batch;
    float scale;
} radon_job_t;

/* Uneven batch (Sec. 4.1 batch processing, for jobs of different image sizes and
 * angle sets): all jobs in ONE persistent kernel launch that pulls work items from a
 * device queue, longest first.  Results equal those of radon_forward /
 * radon_backproject per job bitwise, except the 16-bit forward: it takes horizontal tap
 * pairs with the bilinear weights rounded to the storage type (one dot2 per row and
 * image), so it differs from the per-job forward by that rounding, within the 16-bit
 * error of either against exact arithmetic.  The job table is built and uploaded on
 * the first call for a given job list (by content); later calls with the same list only
 * launch, so the call can be captured into a hipGraph once that first call has run. */
int radon_forward_batched(const radon_job_t *jobs, int32_t n_jobs, int32_t dtype, void *stream);
int radon_backproject_batched(const radon_job_t *jobs, int32_t n_jobs, int32_t dtype,
                              void *stream);

/* Filters of filtered backprojection (Sec. 3.1.3). */
enum { RADON_FILTER_RAMLAK = 0, RADON_FILTER_SHEPP_LOGAN = 1, RADON_FILTER_COSINE = 2,
       RADON_FILTER_HAMMING = 3, RADON_FILTER_HANN = 4 };

/* Sinogram filter of filtered backprojection (Sec. 3.1.3): every projection row of
 * y[batch][A][D] is filtered in the frequency domain by the band-limited ramp whose
 * Fourier filter is built as Kak & Slaney (ch. 3, eq. 61) prescribe -- the transform
 * of the sampled impulse response h(0) = 1/4, h(n) = -1/(pi^2 n^2) for odd n, 0 for
 * even n, over a zero-padded length L = the smallest power of two >= max(64, 2D) --
 * times the window of `filter` at the normalised frequency f in [-1/2, 1/2)
 * (Shepp-Logan sin(pi f)/(pi f), cosine cos(pi f), Hamming 0.54 + 0.46 cos(2 pi f),
 * Hann 0.5 + 0.5 cos(2 pi f), Ram-Lak 1), and scaled by pi / A, so that
 * radon_backproject of the result reconstructs the image when the A angles cover
 * [0, pi) uniformly, at any det_spacing (the sampled kernel's 1/det_spacing cancels
 * the transpose's density of 1/det_spacing bins per unit of detector length).  out may equal y (in place).  FP32 arithmetic for every
 * storage type.  Parallel beam only (RADON_ERR_UNSUPPORTED for the fan beam, and for
 * D > 4096).  Builds its FP32 filter table on first use (RADON_ERR_NOT_PREPARED if
 * that first use is under stream capture). */
int radon_filter_sinogram(const radon_geometry_t *geometry, const void *y, void *out,
                          int32_t batch, int32_t filter, int32_t dtype, void *stream);

/* Library utility (no operation of the paper; the inner products of the conjugate
 * gradient solvers of Sec. 4.2 and 4.3, the adjoint (dot-product) test and losses):
 * FP64 inner product sum_i a[i]*b[i] over n elements of `dtype` (device pointers),
 * written to out (device, one double).  Deterministic (fixed reduction tree).  Uses
 * library-owned partials, one set per (device, stream), so calls on different streams
 * may overlap; the first call on a device must not be under stream capture
 * (RADON_ERR_NOT_PREPARED). */
int radon_dot_f64(const void *a, const void *b, int64_t n, int32_t dtype, double *out,
                  void *stream);

/* ---------------------------------------------------------------- shearlets
 * Alpha-shearlet transform (Sec. 2.1 lists it among the GPU routines; Sec. 3.2 uses
 * real-valued alpha-shearlets, alpha = 0.5, 5 scales, normalised on the Fourier side
 * to a Parseval frame, 59 channels for a 512 x 512 image).  The Fourier filters psi_m
 * of the system are built once per (device, shape, alphas) in FP64 on the host and
 * kept in FP32 on the device; every transform is FFTs and products on the GPU:
 *   forward  c[b][m] = Re IFFT2(FFT2(x[b]) psi_m)
 *   adjoint  x[b]    = Re IFFT2(sum_m FFT2(c[b][m]) psi_m)  (adjoint(forward(x)) = x)
 * The system: r = max(|xi_1|, |xi_2|) of the frequency in cycles per sample; a smooth
 * low-pass and J radial bands (plateau of the low-pass up to 2^-(J+1)); per scale j,
 * ceil(2^(j (1 - alpha_j))) shears on each side of the centre in each of the two
 * frequency cones, with angular windows whose squares sum to 1; the squares of all
 * filters sum to 1 at every frequency.  Channel order: the low-pass, then per scale
 * the horizontal cone's shears -K..K and the vertical cone's -K..K. */
typedef struct radon_shearlet {
    int32_t width;            /* W, a power of two in [16, 4096] (RADON_ERR_UNSUPPORTED otherwise) */
    int32_t height;           /* H, a power of two in [16, 4096] */
    int32_t n_scales;         /* J in [1, 16] */
    int32_t reserved;         /* 0 */
    const double *alphas;     /* host [J], each in [0, 1]; read during the call */
} radon_shearlet_t;

/* Number of coefficient channels M of the system (Sec. 3.2: 59 for 512 x 512, five
 * scales of alpha = 0.5), or a negative status.  Host only. */
int radon_shearlet_channels(const radon_shearlet_t *s);

/* Scale of every channel (Sec. 3.2's regularised reconstruction weighs channels by
 * scale): scales[0] = 0 for the low-pass, j + 1 for the channels of scale j.  scales:
 * host array of radon_shearlet_channels(s) entries.  Host only. */
int radon_shearlet_scales(const radon_shearlet_t *s, int32_t *scales);

/* Library utility (prepares the transforms of Sec. 3.2): build the filters of s on the
 * current device and grow the null stream's workspace for `batch` images (call before
 * capturing a stream that will use s; synchronises the device). */
int radon_shearlet_prepare(const radon_shearlet_t *s, int32_t batch);

/* Forward alpha-shearlet transform (Sec. 2.1, 3.2): coeffs[b][m][H][W] for the images
 * x[b][H][W], b < batch, m < M.  x, coeffs: device, `dtype` (FP32, FP16 or BF16
 * storage; FP32 arithmetic), contiguous, 16-byte aligned.  Uses the stream's library
 * workspace (up to ~0.6 GB; RADON_ERR_NOT_PREPARED if it must grow under capture).
 * Asynchronous on `stream`. */
int radon_shearlet_forward(const radon_shearlet_t *s, const void *x, void *coeffs, int32_t batch,
                           int32_t dtype, void *stream);

/* Adjoint (and, the frame being Parseval, inverse) of radon_shearlet_forward (Sec.
 * 3.2): x[b][H][W] from coeffs[b][m][H][W].  Same layouts, ownership and errors. */
int radon_shearlet_adjoint(const radon_shearlet_t *s, const void *coeffs, void *x, int32_t batch,
                           int32_t dtype, void *stream);

/* ---------------------------------------------------------------- solvers
 * Iterative reconstruction with the projector pair (TorchRadon Sec. 4.2: Landweber
 * iteration and conjugate gradient on the normal equations; Sec. 4.3: conjugate
 * gradient for a symmetric positive definite operator).  A batch holds independent
 * systems stored one after another; every system has its own step sizes.  Scalars stay
 * in device memory, so a solve is queued on the stream without waiting on the host. */

/* Per-system FP64 inner products of the conjugate-gradient solvers (Sec. 4.2, 4.3):
 * out[k] = sum_{i<n} a[k n + i] * b[k n + i] for
 * k < batch (a, b: device, `dtype`, 16-byte aligned; out: device, batch doubles).
 * Deterministic (fixed reduction tree).  batch <= 65535, else RADON_ERR_INVALID_ARG;
 * n == 0 writes zeros.  Uses a library-owned partials buffer per (device, stream),
 * so calls on different streams may overlap; it is grown outside stream capture
 * (RADON_ERR_NOT_PREPARED if it must be created or grown under capture: call once on
 * the capturing stream before capturing). */
int radon_dot_f64_batched(const void *a, const void *b, int64_t n, int32_t batch, int32_t dtype,
                          double *out, void *stream);

/* For callers that cannot allocate (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): radon_dot_f64_batched with no allocation at any
 * call.  Same arguments, layouts, errors and results (the same kernels and reduction
 * tree, so bit for bit the same values).  The partial sums live in a fixed array of
 * 65536 doubles (512 KiB) of device memory that every GPU the library runs on holds
 * until the process ends; a call needs batch * c of them, c = min(64, max(1,
 * ceil(n / 4096))), and returns RADON_ERR_SCRATCH without launching anything when
 * that exceeds 65536 (e.g. more than 1024 systems of >= 258048 elements).  Every call
 * on one GPU uses that GPU's one array: calls that overlap on a GPU (two streams, or
 * two threads) race and give wrong results, so serialise them.  The first call on a
 * device looks the array's address up (no allocation). */
int radon_dot_f64_batched_noalloc(const void *a, const void *b, int64_t n, int32_t batch,
                                  int32_t dtype, double *out, void *stream);

/* Per-system scaled update of the solvers (Sec. 4.2, 4.3): out[k n + i] = u[k n + i] + c_k v[k n + i] with
 * c_k = c0 * num[k] / den[k] evaluated in FP64 (num or den NULL reads as 1; c_k = 0
 * where den[k] == 0, which freezes a system whose search direction has vanished).
 * The element arithmetic is FP64, rounded once to FP32 and then to `dtype`.  Where
 * c_k == 0 the output is u exactly and v is not read.  out may equal u or v.
 * u, v, out: device, `dtype`, 16-byte aligned; num, den: device doubles (8-byte
 * aligned) or NULL.  batch <= 65535. */
int radon_axpy_ratio(const void *u, const void *v, void *out, const double *num,
                     const double *den, double c0, int64_t n, int32_t batch, int32_t dtype,
                     void *stream);

enum { RADON_SOLVER_LANDWEBER = 0, RADON_SOLVER_CGNE = 1 };

/* Library utility (workspace size of the solvers of Sec. 4.2): bytes of workspace
 * radon_landweber (RADON_SOLVER_LANDWEBER) or radon_cgne
 * (RADON_SOLVER_CGNE) needs for `batch` systems of this geometry and dtype; negative
 * status on a bad argument. */
int64_t radon_solver_workspace_bytes(const radon_geometry_t *geometry, int32_t solver,
                                     int32_t batch, int32_t dtype);

/* Landweber iteration (Sec. 4.2) x <- x - alpha R^T (R x - y), `iterations` times, in place on x
 * [batch][N][N] (device, the initial guess on entry); y [batch][A][D] (device).
 * alpha is applied inside the backprojection kernel (no unscaled gradient is stored).
 * workspace: device, 16-byte aligned, at least radon_solver_workspace_bytes(...,
 * RADON_SOLVER_LANDWEBER, ...) bytes, owned by the caller and not used after the
 * queued work completes.  Any dtype.  Status codes as radon_forward. */
int radon_landweber(const radon_geometry_t *geometry, const void *y, void *x, int32_t batch,
                    double alpha, int32_t iterations, int32_t dtype, void *workspace,
                    int64_t workspace_bytes, void *stream);

/* Conjugate gradient on the normal equations R^T R x = R^T y (CGNE, TorchRadon
 * Sec. 4.2), `iterations` steps from the guess in x, in place, every batch entry its
 * own system: r = y - R x, s = R^T r, p = s; then per step q = R p,
 * a = <s,s>/<q,q>, x += a p, r -= a q, s' = R^T r, p = s' + (<s',s'>/<s,s>) p.  Inner
 * products in FP64 (radon_dot_f64_batched), updates by radon_axpy_ratio, so a system
 * whose normal-equation residual reaches exactly zero stays where it is.  FP32 only
 * (RADON_ERR_UNSUPPORTED otherwise: R^T r is stored unscaled).  workspace as for
 * radon_landweber with RADON_SOLVER_CGNE.  Status codes as radon_forward. */
int radon_cgne(const radon_geometry_t *geometry, const void *y, void *x, int32_t batch,
               int32_t iterations, int32_t dtype, void *workspace, int64_t workspace_bytes,
               void *stream);

/* Library utility (no operation of the paper): calibration of the current device for
 * roofline fractions: the FP32 multiply-add
 * rate (multiply-adds per second, v_fmac_f32 with packed FP32 off, many independent
 * chains) and the LDS read bandwidth (bytes per second, conflict-free 16-byte reads)
 * that two fixed-length microbenchmark kernels reach; best of three timed runs after a
 * warm-up run.  Host outputs.  Synchronises the null stream; allocates and frees a small
 * device buffer.  RADON_ERR_INVALID_ARG for a null output. */
int radon_measure_peaks(double *fma_per_s, double *lds_bytes_per_s);

/* Library utility (no operation of the paper): free every plan, table, workspace and
 * scratch buffer the library holds (synchronises the device).  Graphs captured
 * before must not be replayed afterwards. */
int radon_release_plans(void);

/* Library utility (no operation of the paper): launch shape chosen for a
 * geometry/dtype/batch (after radon_prepare):
 * out[0..4] = forward {images per thread, angles per work item, staging, variant,
 * slab rows}, out[5..9] = backprojection {images per thread, angles per LDS block,
 * staging, variant, tile side in pixels}.  variant: 0 = direct kernel, 1 = tiled
 * kernel.  staging: 1 when the tiled kernel first copies the call's input (images,
 * or sinograms for the backprojection) into a zero-bordered, image-interleaved
 * workspace; 2 (16-bit storage) when that copy holds pairs of neighbouring pixels
 * (bins) and each pair of taps is applied by one FP32-accumulating dot2 instruction
 * with the weights rounded to the storage type; else 0.  Builds the plan when
 * missing; status codes as radon_forward. */
int radon_plan_info(const radon_geometry_t *geometry, int32_t dtype, int32_t batch,
                    int32_t *out10);

/* Library utility (no operation of the paper): static description of a status code. */
const char *radon_status_string(int status);

/* Library utility (no operation of the paper): version, major*10000 + minor*100 +
 * patch. */
int radon_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RADON_H */
