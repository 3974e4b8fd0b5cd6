"""GPU parity: the HIP forward projection and backprojection against the FP64 oracle.

Bars: relative L2 <= 1e-5 for FP32 storage; <= 5e-3 for FP16/BF16 storage against
the oracle on the original FP32 inputs (storage rounding included).  Every case
prints its error line ("[parity] ...").
"""
import math

import numpy as np
import pytest

import oracle
from paper_2009_14788_amd import inputs
from _helpers import Case, TOL_16, TOL_F32, rel_l2, max_rel, report, sample_indices, workload_case

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def _dev(a, dt="f32"):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda").to(TDT[dt])


def _host(t):
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def _announce(name, case, dt, batch):
    print(f"[gpu-step] {name} {case!r} dtype={dt} batch={batch}", flush=True)


def _full_check(name, case, x, dt="f32", tol=TOL_F32, y_seed=None):
    """Full-tensor comparison of forward and backprojection for the batch x."""
    op = case.library()
    og = case.oracle()
    B = x.shape[0]
    _announce(name + ":forward", case, dt, B)
    y_gpu = _host(op.forward(_dev(x, dt)))
    y_ref = oracle.forward(og, x)
    e_fwd = rel_l2(y_gpu, y_ref)
    # backprojection of an independent sinogram (N(0,1)) and of the forward result
    ys = inputs.randn(y_ref.shape, 1000 if y_seed is None else y_seed, np.float64)
    _announce(name + ":backprojection", case, dt, B)
    xb_gpu = _host(op.backprojection(_dev(ys, dt)))
    xb_ref = oracle.backproject(og, ys)
    e_bp = rel_l2(xb_gpu, xb_ref)
    report(name, dtype=dt, fwd_rel_l2=e_fwd, fwd_max_rel=max_rel(y_gpu, y_ref),
           bp_rel_l2=e_bp, bp_max_rel=max_rel(xb_gpu, xb_ref))
    assert e_fwd <= tol, (name, "forward", e_fwd)
    assert e_bp <= tol, (name, "backprojection", e_bp)
    return e_fwd, e_bp


# ------------------------------------------------------------------ small full cases
def test_single64_parallel():
    w = inputs.WORKLOADS["single64"]
    x = inputs.phantom(64, 10, [0, 0])[0][None].astype(np.float64)
    _full_check("single64", workload_case(w), x)


def test_single64_fanbeam():
    case = Case("fanbeam", 64, inputs.uniform_angles(64, 2 * math.pi), 91, 1.5, 120.0, 60.0)
    x = inputs.phantom(64, 10, [0, 1])[0][None].astype(np.float64)
    _full_check("single64_fan", case, x)


@pytest.mark.parametrize("beam", ["parallel", "fanbeam"])
def test_ragged_geometry(beam):
    """Odd sizes and a ragged batch (5 images over 4-image groups), arbitrary angles
    (negative, beyond 2 pi, exact axes), spacing 0.8 and step 0.7."""
    ang = [-0.3, 0.0, math.pi / 2, 1.234, 3 * math.pi, 7.5, -2.0]
    if beam == "parallel":
        case = Case(beam, 37, ang, 53, 0.8, step=0.7)
    else:
        case = Case(beam, 37, ang, 53, 1.3, 70.0, 31.0, step=0.7)
    x = inputs.randn((5, 37, 37), 17, np.float64)
    _full_check("ragged_" + beam, case, x)


@pytest.mark.parametrize("beam", ["parallel", "fanbeam"])
def test_degenerate_sizes(beam):
    """N = 1 (a single pixel), D = 1, A = 1, and D much wider than the image."""
    for n, ang, D in [(1, [0.3], 1), (1, [0.0, 1.0, 2.0], 5), (2, [0.7], 1), (5, [0.0], 40)]:
        case = (Case(beam, n, ang, D, 1.0) if beam == "parallel"
                else Case(beam, n, ang, D, 1.0, 10.0, 4.0))
        x = inputs.randn((3, n, n), 5, np.float64)
        _full_check(f"degenerate_{beam}_n{n}_d{D}", case, x)


def test_batch16_256_parallel():
    """16 x 256^2, 256 angles, 363 bins: full GPU batch; oracle on 3 whole images
    plus sampled rays and pixels of the rest."""
    w = inputs.WORKLOADS["batch16_256"]
    case = workload_case(w)
    x = inputs.phantom_batch(1, 16, 256).astype(np.float64)
    op, og = case.library(), case.oracle()
    _announce("batch16_256:forward", case, "f32", 16)
    y_gpu = _host(op.forward(_dev(x)))
    y_ref3 = oracle.forward(og, x[:3])
    e_full = rel_l2(y_gpu[:3], y_ref3)
    rng = np.random.default_rng(123)
    idx = sample_indices(rng, 400, (16, w.n_angles, w.det_count))
    e_samp = rel_l2(y_gpu[idx[:, 0], idx[:, 1], idx[:, 2]], oracle.forward_rays(og, x, idx))
    ys = inputs.randn((16, w.n_angles, w.det_count), 99, np.float64)
    _announce("batch16_256:backprojection", case, "f32", 16)
    xb_gpu = _host(op.backprojection(_dev(ys)))
    xb_ref2 = oracle.backproject(og, ys[:2])
    e_bfull = rel_l2(xb_gpu[:2], xb_ref2)
    pidx = sample_indices(rng, 48, (16, 256, 256))
    e_bsamp = rel_l2(xb_gpu[pidx[:, 0], pidx[:, 1], pidx[:, 2]],
                     oracle.backproject_pixels(og, ys, pidx))
    report("batch16_256", fwd_rel_l2_img0to2=e_full, fwd_rel_l2_sampled=e_samp,
           bp_rel_l2_img0to1=e_bfull, bp_rel_l2_sampled=e_bsamp)
    assert max(e_full, e_samp, e_bfull, e_bsamp) <= TOL_F32


# ------------------------------------------------------------------ headline size, sampled
def _sampled_check(name, case, x, dt, tol, n_rays=256, n_pix=32, seed=7):
    """Sampled outputs at full size, in the launch shapes the autotuner picks for this
    batch (the configuration the benchmark times)."""
    op, og = case.library(), case.oracle()
    B = x.shape[0]
    op.prepare(TDT[dt], B)
    shapes = op.plan_info(TDT[dt], B)
    _announce(name + ":forward", case, dt, B)
    y_gpu = op.forward(_dev(x, dt))
    rng = np.random.default_rng(seed)
    idx = sample_indices(rng, n_rays, (B, case.angles.size, case.det_count))
    yg = _host(y_gpu[idx[:, 0], idx[:, 1], idx[:, 2]])
    del y_gpu
    e_fwd = rel_l2(yg, oracle.forward_rays(og, x, idx))
    ys = inputs.randn((B, case.angles.size, case.det_count), seed + 1, np.float32)
    _announce(name + ":backprojection", case, dt, B)
    xb = op.backprojection(_dev(ys, dt))
    pidx = sample_indices(rng, n_pix, (B, case.n, case.n))
    xg = _host(xb[pidx[:, 0], pidx[:, 1], pidx[:, 2]])
    del xb
    e_bp = rel_l2(xg, oracle.backproject_pixels(og, ys.astype(np.float64), pidx))
    report(name, dtype=dt, fwd_rel_l2_sampled=e_fwd, bp_rel_l2_sampled=e_bp,
           rays=n_rays, pixels=n_pix, shapes=shapes)
    assert e_fwd <= tol and e_bp <= tol, (e_fwd, e_bp)


def test_headline_batch128_512_sampled():
    """128 x 512^2, 720 angles over [0, pi), 724 bins (the benchmark workload), FP32,
    in the launch configuration the benchmark times."""
    w = inputs.WORKLOADS["batch128_512"]
    x = inputs.phantom_batch(2, 128, 512).astype(np.float64)
    _sampled_check("batch128_512", workload_case(w), x, "f32", TOL_F32)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_fan64_512_sampled(dt):
    """64 x 512^2 fan beam, S = 1000, E = 500, 1024 bins x 1.5, 1024 angles over
    [0, 2 pi), 16-bit storage with FP32 accumulation."""
    w = inputs.WORKLOADS["fan64_512"]
    x = inputs.phantom_batch(4, 64, 512).astype(np.float64)
    # the oracle sees the original FP32 values: the bar includes storage rounding
    _sampled_check("fan64_512", workload_case(w), x, dt, TOL_16, n_rays=256, n_pix=24)


# ------------------------------------------------------------------ 16-bit storage
@pytest.mark.parametrize("dt", ["f16", "bf16"])
@pytest.mark.parametrize("beam", ["parallel", "fanbeam"])
def test_16bit_storage_small(dt, beam):
    """FP16/BF16 storage, FP32 accumulation: error against the oracle on the FP32
    inputs (bar 5e-3), and against the oracle on the 16-bit-rounded inputs (kernel
    arithmetic only; FP32-level agreement up to the output rounding)."""
    if beam == "parallel":
        case = Case(beam, 128, inputs.uniform_angles(96), 182, 1.0)
    else:
        case = Case(beam, 128, inputs.uniform_angles(96, 2 * math.pi), 160, 1.5, 250.0, 125.0)
    x = inputs.phantom_batch(5, 3, 128).astype(np.float64)
    _full_check(f"storage_{dt}_{beam}", case, x, dt, TOL_16)
    # secondary: inputs rounded to the storage type first
    op, og = case.library(), case.oracle()
    xr = _dev(x, dt)
    y_gpu = _host(op.forward(xr))
    y_ref = oracle.forward(og, _host(xr))
    out_ulp = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[dt]
    e = rel_l2(y_gpu, y_ref)
    report(f"storage_{dt}_{beam}_rounded_inputs", fwd_rel_l2=e)
    assert e <= out_ulp


def test_fp16_backprojection_overflow_is_inf():
    """FP16 outputs beyond 65504 are stored as +inf (documented behaviour)."""
    case = Case("parallel", 16, inputs.uniform_angles(64), 23)
    op = case.library()
    y = torch.full((1, 64, 23), 60000.0, device="cuda", dtype=torch.float16)
    xb = op.backprojection(y)
    torch.cuda.synchronize()
    assert torch.isinf(xb).any().item()
    # scaled down, the same call is finite
    xs = op.backprojection(y, scale=1e-3)
    assert torch.isfinite(xs).all().item()


def test_scale_argument():
    case = Case("parallel", 32, inputs.uniform_angles(20), 46)
    op = case.library()
    x = _dev(inputs.randn((2, 32, 32), 3))
    y1 = op.forward(x)
    y2 = op.forward(x, scale=-2.5)
    torch.cuda.synchronize()
    assert torch.allclose(y2, -2.5 * y1, rtol=1e-6, atol=1e-6)


def test_batch_zero_and_shapes():
    case = Case("parallel", 16, inputs.uniform_angles(8), 23)
    op = case.library()
    out = op.forward(torch.empty((0, 16, 16), device="cuda"))
    assert out.shape == (0, 8, 23)
    y = op.forward(_dev(inputs.randn((16, 16), 1)))
    assert y.shape == (8, 23)
    y3 = op.forward(_dev(inputs.randn((2, 3, 16, 16), 1)))
    assert y3.shape == (2, 3, 8, 23)


# ------------------------------------------------------------------ adjointness on the GPU
@pytest.mark.parametrize("beam", ["parallel", "fanbeam"])
def test_dot_product_gpu(beam):
    """<R x, y> = <x, R^T y> with the GPU kernels and FP64 GPU reductions,
    32 x 32 images, 48 angles, 46 bins, N(0,1) x and y: relative gap <= 1e-6."""
    from paper_2009_14788_amd.radon import dot_f64
    if beam == "parallel":
        case = Case(beam, 32, inputs.uniform_angles(48), 46)
    else:
        case = Case(beam, 32, inputs.uniform_angles(48, 2 * math.pi), 46, 2.0, 80.0, 40.0)
    op = case.library()
    x = _dev(inputs.randn((4, 32, 32), 7))
    y = _dev(inputs.randn((4, 48, 46), 8))
    lhs = dot_f64(op.forward(x), y).item()
    rhs = dot_f64(x, op.backprojection(y)).item()
    gap = abs(lhs - rhs) / max(abs(lhs), abs(rhs))
    report(f"dot_{beam}", gap=gap, lhs=lhs, rhs=rhs)
    assert gap <= 1e-6
