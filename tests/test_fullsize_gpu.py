"""Full-size parity against the FP64 oracle, in the launch shapes the benchmark times.

Every element of every image is compared, per image (a fault confined to one image,
lane or LDS plane position cannot hide in an average):

* 128 x 512^2, 720 angles over [0, pi), 724 bins, FP32 / FP16 / BF16 storage after
  prepare(dtype, 128) -- both directions, all 128 images;
* 64 x 512^2 fan beam (S = 1000, E = 500, 1024 bins x 1.5, 1024 angles over
  [0, 2 pi)), BF16 / FP16 storage, both directions, all 64 images;
* the 200-job uneven batch in one persistent launch, FP32 / FP16, eager and
  graph-replayed, every job whole, both directions;
* the 64-images-per-lane backprojection (single-level FP32 sums) at 2048 angles;
* the 16-bit tap-pair shapes (dot2 with 16-bit weights) in both directions, forced,
  at the headline and fan-beam sizes.

Bars: relative L2 <= 1e-5 (FP32) and <= 5e-3 (16-bit storage, against the oracle on
the original FP32 inputs, storage rounding included) for every image.  Each case
prints "[parity] ..." lines with the overall and worst per-image relative L2 and
max|err| / max|ref|.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2009_14788_amd import inputs
from _helpers import Case, TOL_16, TOL_F32, max_rel, rel_l2, report, workload_case

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
TOL = {"f32": TOL_F32, "f16": TOL_16, "bf16": TOL_16}
# images at every lane and plane position of the 4-, 8-, 16- and 64-image groups
POSITIONS = (0, 3, 4, 7, 8, 15, 16, 31, 32, 63, 64, 100, 126, 127)


def _announce(msg):
    print(f"[gpu-step] {msg}", flush=True)


def _host(t):
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def per_image_rel_l2(got, ref):
    g = got.reshape(got.shape[0], -1)
    r = ref.reshape(ref.shape[0], -1)
    den = np.linalg.norm(r, axis=1)
    return np.linalg.norm(g - r, axis=1) / np.where(den > 0, den, 1.0)


def _compare(tag, got, ref, tol, **extra):
    e_img = per_image_rel_l2(got, ref)
    e_all = rel_l2(got, ref)
    worst = int(np.argmax(e_img))
    report(tag, rel_l2=e_all, worst_image_rel_l2=float(e_img[worst]), worst_image=worst,
           max_abs_over_max_ref=max_rel(got, ref), images=got.shape[0], **extra)
    assert np.all(e_img <= tol), (tag, worst, float(e_img[worst]))
    return e_all, float(e_img[worst])


# ------------------------------------------------------------------ headline 128 x 512^2
@pytest.fixture(scope="module")
def headline():
    w = inputs.WORKLOADS["batch128_512"]
    case = workload_case(w)
    og = case.oracle()
    x = inputs.phantom_batch(2, w.batch, w.n)                      # the benchmark's phantoms
    ys = inputs.randn((w.batch, w.n_angles, w.det_count), 2024)    # N(0,1) sinograms
    _announce("oracle forward + backprojection, 128 x 512^2, 720 angles, 724 bins")
    y_ref = oracle.forward(og, x.astype(np.float64))
    xb_ref = oracle.backproject(og, ys.astype(np.float64))
    return case, og, x, ys, y_ref, xb_ref


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_headline_full(headline, dt):
    case, og, x, ys, y_ref, xb_ref = headline
    op = case.library()
    B = x.shape[0]
    op.prepare(TDT[dt], B)
    shapes = op.plan_info(TDT[dt], B)
    _announce(f"headline forward {dt} batch {B} shapes {shapes}")
    xd = torch.from_numpy(x).cuda().to(TDT[dt])
    y_gpu = _host(op.forward(xd))
    _compare(f"headline_fwd_{dt}", y_gpu, y_ref, TOL[dt], shape=shapes["forward"])
    if dt != "f32":
        # kernel arithmetic alone: the oracle on the 16-bit-rounded images, at every
        # lane and plane position; the outputs differ by at most their own rounding
        sel = list(POSITIONS)
        xr = _host(xd[sel])
        ref_r = oracle.forward(og, xr)
        e = rel_l2(y_gpu[sel], ref_r)
        report(f"headline_fwd_{dt}_rounded_inputs", rel_l2=e, images=len(sel))
        assert e <= {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[dt]
    del y_gpu, xd
    _announce(f"headline backprojection {dt} batch {B}")
    yd = torch.from_numpy(ys).cuda().to(TDT[dt])
    xb_gpu = _host(op.backprojection(yd))
    _compare(f"headline_bp_{dt}", xb_gpu, xb_ref, TOL[dt], shape=shapes["backprojection"])
    if dt != "f32":
        sel = list(POSITIONS)
        yr = _host(yd[sel])
        ref_r = oracle.backproject(og, yr)
        e = rel_l2(xb_gpu[sel], ref_r)
        report(f"headline_bp_{dt}_rounded_inputs", rel_l2=e, images=len(sel))
        assert e <= {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[dt]


class _forced_shape:
    """RADON_FORCE_SHAPE for the calls inside the block (read at every call)."""

    def __init__(self, shape):
        self.shape, self.old = shape, None

    def __enter__(self):
        self.old = os.environ.get("RADON_FORCE_SHAPE")
        os.environ["RADON_FORCE_SHAPE"] = self.shape

    def __exit__(self, *exc):
        if self.old is None:
            os.environ.pop("RADON_FORCE_SHAPE", None)
        else:
            os.environ["RADON_FORCE_SHAPE"] = self.old


def _pairs_case(tag, op, og, x, ys, y_ref, xb_ref, dt, shape):
    """Both directions in a forced shape (mostly tap-pair staging: 16-bit weights,
    dot2), whatever the autotuner picks: every image against the oracle on the FP32
    inputs, and the kernel arithmetic alone (the oracle on the 16-bit-rounded inputs)
    at every lane and plane position."""
    with _forced_shape(shape):
        _announce(f"{tag} tap pairs {dt} shape {shape}")
        xd = torch.from_numpy(x).cuda().to(TDT[dt])
        y_gpu = _host(op.forward(xd))
        _compare(f"{tag}_fwd_pairs_{dt}", y_gpu, y_ref, TOL[dt], shape=shape)
        sel = [p for p in POSITIONS if p < x.shape[0]]
        e = rel_l2(y_gpu[sel], oracle.forward(og, _host(xd[sel])))
        report(f"{tag}_fwd_pairs_{dt}_rounded_inputs", rel_l2=e, images=len(sel))
        assert e <= {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[dt]
        del y_gpu, xd
        yd = torch.from_numpy(ys).cuda().to(TDT[dt])
        xb_gpu = _host(op.backprojection(yd))
        _compare(f"{tag}_bp_pairs_{dt}", xb_gpu, xb_ref, TOL[dt], shape=shape)
        e = rel_l2(xb_gpu[sel], oracle.backproject(og, _host(yd[sel])))
        report(f"{tag}_bp_pairs_{dt}_rounded_inputs", rel_l2=e, images=len(sel))
        assert e <= {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[dt]


@pytest.mark.parametrize("shape", ["8,2,64,4,2", "16,2,32,8,2"])
@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_headline_tap_pairs(headline, dt, shape):
    case, og, x, ys, y_ref, xb_ref = headline
    _pairs_case("headline", case.library(), og, x, ys, y_ref, xb_ref, dt, shape)


# ------------------------------------------------------------------ fan beam 64 x 512^2
@pytest.fixture(scope="module")
def fan():
    w = inputs.WORKLOADS["fan64_512"]
    case = workload_case(w)
    og = case.oracle()
    x = inputs.phantom_batch(4, w.batch, w.n)
    ys = inputs.randn((w.batch, w.n_angles, w.det_count), 4024)
    _announce("oracle fan forward + backprojection, 64 x 512^2, 1024 angles, 1024 bins")
    y_ref = oracle.forward(og, x.astype(np.float64))
    xb_ref = oracle.backproject(og, ys.astype(np.float64))
    return case, og, x, ys, y_ref, xb_ref


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_fan_full(fan, dt):
    case, og, x, ys, y_ref, xb_ref = fan
    op = case.library()
    B = x.shape[0]
    op.prepare(TDT[dt], B)
    shapes = op.plan_info(TDT[dt], B)
    _announce(f"fan forward {dt} batch {B} shapes {shapes}")
    y_gpu = _host(op.forward(torch.from_numpy(x).cuda().to(TDT[dt])))
    _compare(f"fan_fwd_{dt}", y_gpu, y_ref, TOL[dt], shape=shapes["forward"])
    del y_gpu
    _announce(f"fan backprojection {dt} batch {B}")
    xb_gpu = _host(op.backprojection(torch.from_numpy(ys).cuda().to(TDT[dt])))
    _compare(f"fan_bp_{dt}", xb_gpu, xb_ref, TOL[dt], shape=shapes["backprojection"])


@pytest.mark.parametrize("shape", ["16,2,64,4,2", "8,2,32,4,2", "16,2,64,2,2"])
@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_fan_tap_pairs(fan, dt, shape):
    case, og, x, ys, y_ref, xb_ref = fan
    _pairs_case("fan", case.library(), og, x, ys, y_ref, xb_ref, dt, shape)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_fan_two_angle_blocks(fan, dt):
    """Fan backprojection staging two angles per LDS block (interleaved 16-bit copy,
    64 images per lane), every image against the oracle."""
    case, og, x, ys, y_ref, xb_ref = fan
    _pairs_case("fan_ab2", case.library(), og, x, ys, y_ref, xb_ref, dt, "16,1,64,2,1")


# ------------------------------------------------------------------ 200 uneven jobs
@pytest.fixture(scope="module")
def uneven():
    jobs = inputs.uneven_jobs(200)
    xs = [inputs.uneven_phantom(j)[None] for j in jobs]
    gs = [inputs.randn((1, j.n_angles, j.det_count), 5000 + i) for i, j in enumerate(jobs)]
    _announce("oracle forward + backprojection of the 200 uneven jobs")
    y_ref, b_ref = [], []
    for j, x, g in zip(jobs, xs, gs):
        og = Case("parallel", j.n, j.angles(), j.det_count).oracle()
        y_ref.append(oracle.forward(og, x.astype(np.float64)))
        b_ref.append(oracle.backproject(og, g.astype(np.float64)))
    return jobs, xs, gs, y_ref, b_ref


@pytest.mark.parametrize("dt", ["f32", "f16"])
def test_uneven200_full_graph(uneven, dt):
    """All 200 jobs in one persistent launch per direction, eager and from a captured
    graph replayed three times (new eager work and synchronisations between replays):
    every replay equals the eager result bitwise, and every job matches the oracle."""
    from paper_2009_14788_amd.batched import BatchedRadon
    from paper_2009_14788_amd.radon import Radon
    jobs, xs_np, gs_np, y_ref, b_ref = uneven
    ops = [Radon(j.n, j.angles(), j.det_count, 1.0) for j in jobs]
    br = BatchedRadon(ops)
    xs = [torch.from_numpy(x).cuda().to(TDT[dt]) for x in xs_np]
    gs = [torch.from_numpy(g).cuda().to(TDT[dt]) for g in gs_np]
    ys = [torch.empty((1,) + o.sinogram_shape, device="cuda", dtype=TDT[dt]) for o in ops]
    bs = [torch.empty((1,) + o.image_shape, device="cuda", dtype=TDT[dt]) for o in ops]
    _announce(f"uneven200 eager {dt}")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        br.forward(xs, out=ys)
        br.backprojection(gs, out=bs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager_y = [y.clone() for y in ys]
    eager_b = [b.clone() for b in bs]
    worst_f = worst_b = 0.0
    for k in range(len(jobs)):
        worst_f = max(worst_f, rel_l2(_host(eager_y[k]), y_ref[k]))
        worst_b = max(worst_b, rel_l2(_host(eager_b[k]), b_ref[k]))
    report(f"uneven200_{dt}", fwd_worst_job_rel_l2=worst_f, bp_worst_job_rel_l2=worst_b, jobs=len(jobs))
    assert worst_f <= TOL[dt] and worst_b <= TOL[dt], (worst_f, worst_b)
    _announce(f"uneven200 graph capture {dt}")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        br.forward(xs, out=ys)
        br.backprojection(gs, out=bs)
    for rep in range(3):
        for y in ys:
            y.fill_(float("nan"))
        for b in bs:
            b.fill_(float("nan"))
        ops[rep].forward_raw(xs[rep])               # unrelated eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in range(len(jobs)):
            assert torch.equal(ys[k], eager_y[k]), (rep, k, "forward")
            assert torch.equal(bs[k], eager_b[k]), (rep, k, "backprojection")
    report(f"uneven200_{dt}_graph", replays=3, bitwise_equal_to_eager=True)


# ------------------------------------------------------------------ 64-image backprojection
@pytest.mark.parametrize("n_angles", [2048])
def test_bp64_many_angles(n_angles):
    """The 64-images-per-lane backprojection accumulates every angle straight into one
    FP32 sum per pixel and image (no per-block partials); its error at 2048 angles,
    whole images at four lane positions, against the oracle and beside the
    two-level 32-image shape."""
    case = Case("parallel", 512, inputs.uniform_angles(n_angles), 724)
    og = case.oracle()
    op = case.library()
    B = 64
    ys = inputs.randn((B, n_angles, 724), 7000 + n_angles)
    sel = [0, 21, 42, 63]
    _announce(f"oracle backprojection 512^2, {n_angles} angles, images {sel}")
    ref = oracle.backproject(og, ys[sel].astype(np.float64))
    yd = torch.from_numpy(ys).cuda()
    errs = {}
    old = os.environ.get("RADON_FORCE_SHAPE")
    try:
        for bi in (64, 32):
            os.environ["RADON_FORCE_SHAPE"] = f"8,1,{bi},4,1"
            _announce(f"backprojection {n_angles} angles, {bi} images per lane")
            got = _host(op.backprojection(yd)[sel])
            errs[bi] = rel_l2(got, ref)
            e_img = per_image_rel_l2(got, ref)
            report(f"bp{bi}_{n_angles}angles", rel_l2=errs[bi], worst_image_rel_l2=float(e_img.max()),
                   max_abs_over_max_ref=max_rel(got, ref))
            assert np.all(e_img <= TOL_F32)
    finally:
        if old is None:
            os.environ.pop("RADON_FORCE_SHAPE", None)
        else:
            os.environ["RADON_FORCE_SHAPE"] = old
