// Alpha-shearlet transform: Fourier filters built on the host in FP64, per-shape
// plans on the device, and the C ABI (TorchRadon Sec. 2.1 and 3.2: real-valued
// alpha-shearlets normalised on the Fourier side to a Parseval frame, Fourier
// coefficients computed once, every later transform on the GPU for a batch).
//
// The system (the paper prints no construction; this is a cone-adapted alpha-shearlet
// Parseval frame):
//   frequencies xi = (k2 / W, k1 / H) in FFT order, folded to [-1/2, 1/2);
//   r = max(|xi_1|, |xi_2|);  nu(t) = t^4 (35 - 84 t + 70 t^2 - 20 t^3) on [0, 1];
//   phi(r) = 1 on [0, c], cos(pi/2 nu(r / c - 1)) on [c, 2c], 0 beyond; c = 2^-(J+1);
//   scale j < J-1: W_j^2 = phi(r / 2^(j+1))^2 - phi(r / 2^j)^2; scale J-1: 1 - phi(r / 2^(J-1))^2;
//   K_j = ceil(2^(j (1 - alpha_j))) shears per cone, k = -K_j .. K_j;
//   horizontal cone |xi_2| <= |xi_1|, slope t = xi_2 / xi_1; vertical cone the rest,
//   t = xi_1 / xi_2;  V(u) = cos(pi/2 nu(|u|)) on [-1, 1];
//   psi_{j,cone,k} = W_j(r) V(K_j t - k) [cone];  psi_0 = phi(r);
// so the squares of all filters sum to 1 at every frequency.  On an even grid the
// Nyquist row and column are symmetrised, psi[k] <- sqrt((psi[k]^2 + psi[-k]^2) / 2),
// so every filter is even and the coefficients of a real image are real.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/radon.h"
#include "radon_plan.hpp"
#include "radon_shearlet.hpp"

namespace radon {

static double smooth_step(double t) {
    if (t <= 0.0) return 0.0;
    if (t >= 1.0) return 1.0;
    return t * t * t * t * (35.0 - 84.0 * t + 70.0 * t * t - 20.0 * t * t * t);
}

static double profile(double r, double c) {
    if (r <= c) return 1.0;
    if (r >= 2.0 * c) return 0.0;
    return std::cos(0.5 * M_PI * smooth_step(r / c - 1.0));
}

static double window(double u) {
    const double a = std::fabs(u);
    return a >= 1.0 ? 0.0 : std::cos(0.5 * M_PI * smooth_step(a));
}

static int shears(int j, double alpha) {
    return (int)std::ceil(std::pow(2.0, j * (1.0 - alpha)) - 1e-12);
}

int shearlet_channels(const std::vector<double> &alphas, std::vector<int> *scales) {
    int m = 1;
    if (scales) scales->assign(1, 0);
    for (size_t j = 0; j < alphas.size(); ++j) {
        const int n = 2 * (2 * shears((int)j, alphas[j]) + 1);
        m += n;
        if (scales) scales->insert(scales->end(), n, (int)j + 1);
    }
    return m;
}

int shearlet_filters(int width, int height, const std::vector<double> &alphas,
                     std::vector<double> &out) {
    const int J = (int)alphas.size();
    const int M = shearlet_channels(alphas, nullptr);
    const size_t plane = (size_t)width * height;
    out.assign((size_t)M * plane, 0.0);
    const double c = std::ldexp(1.0, -(J + 1));
    for (int k1 = 0; k1 < height; ++k1) {
        const double x2 = (k1 < (height + 1) / 2 ? k1 : k1 - height) / (double)height;
        for (int k2 = 0; k2 < width; ++k2) {
            const double x1 = (k2 < (width + 1) / 2 ? k2 : k2 - width) / (double)width;
            const double a1 = std::fabs(x1), a2 = std::fabs(x2);
            const double r = std::max(a1, a2);
            const bool horizontal = a2 <= a1;
            const double t = horizontal ? (a1 > 0.0 ? x2 / x1 : 0.0) : x1 / x2;
            const size_t at = (size_t)k1 * width + k2;
            out[at] = profile(r, c);
            size_t m = 1;
            for (int j = 0; j < J; ++j) {
                const int K = shears(j, alphas[j]);
                const double lo = profile(r / std::ldexp(1.0, j), c);
                const double w2 = j < J - 1 ? profile(r / std::ldexp(1.0, j + 1), c) * profile(r / std::ldexp(1.0, j + 1), c) - lo * lo
                                            : 1.0 - lo * lo;
                const double Wj = std::sqrt(std::max(w2, 0.0));
                for (int cone = 0; cone < 2; ++cone) {
                    const bool mine = (cone == 0) == horizontal;
                    for (int k = -K; k <= K; ++k, ++m)
                        if (mine && Wj > 0.0) out[m * plane + at] = Wj * window(K * t - k);
                }
            }
        }
    }
    // even symmetry on the grid: only the Nyquist row / column change
    std::vector<double> f(plane);
    for (int m = 0; m < M; ++m) {
        double *p = out.data() + (size_t)m * plane;
        std::memcpy(f.data(), p, plane * sizeof(double));
        for (int k1 = 0; k1 < height; ++k1)
            for (int k2 = 0; k2 < width; ++k2) {
                const double a = f[(size_t)k1 * width + k2];
                const double b = f[(size_t)((height - k1) % height) * width + (width - k2) % width];
                p[(size_t)k1 * width + k2] = std::sqrt(0.5 * (a * a + b * b));
            }
    }
    return M;
}

// ---------------------------------------------------------------- plans
struct ShearletPlan {
    ShearletDims dims;
    float2 *psi = nullptr;
    float2 *tw_w = nullptr;
    float2 *tw_h = nullptr;
    ShearletPlan() = default;
    ShearletPlan(const ShearletPlan &) = delete;
    ShearletPlan &operator=(const ShearletPlan &) = delete;
    ~ShearletPlan() {
        if (psi) (void)hipFree(psi);
        if (tw_w) (void)hipFree(tw_w);
        if (tw_h) (void)hipFree(tw_h);
    }
};

static std::mutex g_sh_mutex;
static std::map<std::tuple<int, int, int, std::vector<double>>, std::unique_ptr<ShearletPlan>> g_sh_plans;

static int log2_exact(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return (1 << l) == v ? l : -1;
}

static int check(const radon_shearlet_t *s) {
    if (!s || !s->alphas) return RADON_ERR_INVALID_ARG;
    if (s->n_scales < 1 || s->n_scales > 16) return RADON_ERR_INVALID_ARG;
    for (int j = 0; j < s->n_scales; ++j)
        if (!std::isfinite(s->alphas[j]) || s->alphas[j] < 0.0 || s->alphas[j] > 1.0)
            return RADON_ERR_INVALID_ARG;
    if (s->width < 1 || s->height < 1) return RADON_ERR_INVALID_ARG;
    const int lw = log2_exact(s->width), lh = log2_exact(s->height);
    if (lw < kShMinLog2 || lw > kShMaxLog2 || lh < kShMinLog2 || lh > kShMaxLog2)
        return RADON_ERR_UNSUPPORTED;
    return RADON_OK;
}

static int twiddles(int n, float2 **out) {
    std::vector<float2> tw(n);
    for (int k = 0; k < n; ++k)
        tw[k] = make_float2((float)std::cos(2.0 * M_PI * k / n), (float)-std::sin(2.0 * M_PI * k / n));
    if (hipMalloc(out, n * sizeof(float2)) != hipSuccess) return RADON_ERR_ALLOC;
    return hipMemcpy(*out, tw.data(), n * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess
               ? RADON_OK : RADON_ERR_HIP;
}

static int shearlet_plan(const radon_shearlet_t *s, hipStream_t stream, ShearletPlan **out) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return RADON_ERR_NO_DEVICE;
    std::vector<double> alphas(s->alphas, s->alphas + s->n_scales);
    auto key = std::make_tuple(device, (int)s->width, (int)s->height, alphas);
    std::lock_guard<std::mutex> lock(g_sh_mutex);
    auto it = g_sh_plans.find(key);
    if (it != g_sh_plans.end()) {
        *out = it->second.get();
        return RADON_OK;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return RADON_ERR_HIP;
    if (cap != hipStreamCaptureStatusNone) return RADON_ERR_NOT_PREPARED;
    std::unique_ptr<ShearletPlan> p(new (std::nothrow) ShearletPlan());
    if (!p) return RADON_ERR_ALLOC;
    std::vector<double> f;
    const int W = s->width, H = s->height;
    const int M = shearlet_filters(W, H, alphas, f);
    ShearletDims &d = p->dims;
    d.log2w = log2_exact(W);
    d.log2h = log2_exact(H);
    d.channels = M;
    d.pairs = (M + 1) / 2;
    // pairs of channels, column-major: psi[p][k2][k1] = (psi_2p, psi_2p+1)[k1][k2]
    const size_t plane = (size_t)W * H;
    std::vector<float2> packed((size_t)d.pairs * plane);
    for (int q = 0; q < d.pairs; ++q)
        for (int k2 = 0; k2 < W; ++k2)
            for (int k1 = 0; k1 < H; ++k1) {
                const size_t at = (size_t)k1 * W + k2;
                const float a = (float)f[(size_t)(2 * q) * plane + at];
                const float b = 2 * q + 1 < M ? (float)f[(size_t)(2 * q + 1) * plane + at] : 0.0f;
                packed[((size_t)q * W + k2) * H + k1] = make_float2(a, b);
            }
    if (hipMalloc(&p->psi, packed.size() * sizeof(float2)) != hipSuccess) return RADON_ERR_ALLOC;
    if (hipMemcpy(p->psi, packed.data(), packed.size() * sizeof(float2), hipMemcpyHostToDevice) !=
        hipSuccess)
        return RADON_ERR_HIP;
    int rc;
    if ((rc = twiddles(W, &p->tw_w)) != RADON_OK || (rc = twiddles(H, &p->tw_h)) != RADON_OK) return rc;
    *out = p.get();
    g_sh_plans.emplace(std::move(key), std::move(p));
    return RADON_OK;
}

static int run_shearlet(const radon_shearlet_t *s, const void *in, void *out, int32_t batch,
                        int32_t dtype, bool adjoint, void *stream) {
    int rc = check(s);
    if (rc != RADON_OK) return rc;
    if (dtype != RADON_F32 && dtype != RADON_F16 && dtype != RADON_BF16) return RADON_ERR_INVALID_ARG;
    if (batch < 0) return RADON_ERR_INVALID_ARG;
    if (batch == 0) return RADON_OK;
    if (!in || !out) return RADON_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) return RADON_ERR_ALIGN;
    hipStream_t st = static_cast<hipStream_t>(stream);
    ShearletPlan *p = nullptr;
    if ((rc = shearlet_plan(s, st, &p)) != RADON_OK) return rc;
    const int chunk = shearlet_chunk(p->dims, batch);
    const size_t need = shearlet_workspace_bytes(p->dims, chunk, adjoint);
    size_t have = 0;
    void *ws = stream_workspace(st, need, &have);
    if (!ws || have < need) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) != hipSuccess) return RADON_ERR_HIP;
        return cap != hipStreamCaptureStatusNone ? RADON_ERR_NOT_PREPARED : RADON_ERR_ALLOC;
    }
    const hipError_t e = launch_shearlet(dtype, adjoint, p->dims, p->psi, p->tw_w, p->tw_h, in, out,
                                         batch, ws, st);
    return e == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

void release_shearlet_plans() {
    std::lock_guard<std::mutex> lock(g_sh_mutex);
    g_sh_plans.clear();
}

}  // namespace radon

using namespace radon;

extern "C" {

int radon_shearlet_channels(const radon_shearlet_t *s) {
    const int rc = check(s);
    if (rc != RADON_OK) return rc;
    return shearlet_channels(std::vector<double>(s->alphas, s->alphas + s->n_scales), nullptr);
}

int radon_shearlet_scales(const radon_shearlet_t *s, int32_t *scales) {
    const int rc = check(s);
    if (rc != RADON_OK) return rc;
    if (!scales) return RADON_ERR_INVALID_ARG;
    std::vector<int> sc;
    shearlet_channels(std::vector<double>(s->alphas, s->alphas + s->n_scales), &sc);
    for (size_t m = 0; m < sc.size(); ++m) scales[m] = sc[m];
    return RADON_OK;
}

int radon_shearlet_prepare(const radon_shearlet_t *s, int32_t batch) {
    int rc = check(s);
    if (rc != RADON_OK) return rc;
    if (batch < 0) return RADON_ERR_INVALID_ARG;
    ShearletPlan *p = nullptr;
    if ((rc = shearlet_plan(s, nullptr, &p)) != RADON_OK) return rc;
    if (batch > 0) {
        const int chunk = shearlet_chunk(p->dims, batch);
        const size_t need = std::max(shearlet_workspace_bytes(p->dims, chunk, false),
                                     shearlet_workspace_bytes(p->dims, chunk, true));
        size_t have = 0;
        if (!stream_workspace(nullptr, need, &have) || have < need) return RADON_ERR_ALLOC;
    }
    return hipDeviceSynchronize() == hipSuccess ? RADON_OK : RADON_ERR_HIP;
}

int radon_shearlet_forward(const radon_shearlet_t *s, const void *x, void *coeffs, int32_t batch,
                           int32_t dtype, void *stream) {
    return run_shearlet(s, x, coeffs, batch, dtype, false, stream);
}

int radon_shearlet_adjoint(const radon_shearlet_t *s, const void *coeffs, void *x, int32_t batch,
                           int32_t dtype, void *stream) {
    return run_shearlet(s, coeffs, x, batch, dtype, true, stream);
}

}  // extern "C"
