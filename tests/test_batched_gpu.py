"""Uneven batches in one persistent launch: identical to per-job calls (the 16-bit forward
within 1e-3 of them), matching the oracle, and replayable from a captured graph."""
import math

import numpy as np
import pytest

import oracle
from paper_2009_14788_amd import inputs
from _helpers import Case, TOL_F32, TOL_16, rel_l2, report, sample_indices

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def _jobs(count, seed=3):
    return inputs.uneven_jobs(count, seed)


def _ops(jobs):
    from paper_2009_14788_amd.radon import Radon
    return [Radon(j.n, j.angles(), j.det_count, 1.0) for j in jobs]


def _images(jobs, dt="f32", batch=1):
    out = []
    for j in jobs:
        x = np.stack([inputs.uneven_phantom(j)] * batch) if batch > 1 else inputs.uneven_phantom(j)[None]
        out.append(torch.from_numpy(x).cuda().to(TDT[dt]))
    return out


@pytest.mark.parametrize("dt", ["f32", "f16"])
def test_batched_equals_per_job(dt):
    """24 jobs from the uneven distribution (N in {128..512}, 30..360 angles over pi or
    2pi/3): the batched forward and backprojection equal the per-job calls bitwise, except
    the 16-bit forward, which takes tap pairs along x (its weights rounded to FP16) and is
    held within 1e-3 of the per-job forward (both are within ~3e-4 of the oracle)."""
    from paper_2009_14788_amd.batched import BatchedRadon
    jobs = _jobs(24)
    ops = _ops(jobs)
    br = BatchedRadon(ops)
    xs = _images(jobs, dt)
    print(f"[gpu-step] batched forward, 24 jobs, {dt}", flush=True)
    ys = br.forward(xs)
    ys_ref = [op.forward_raw(x) for op, x in zip(ops, xs)]
    gs = [torch.randn(op.sinogram_shape, generator=torch.Generator().manual_seed(i)).cuda().to(TDT[dt])[None]
          for i, op in enumerate(ops)]
    print(f"[gpu-step] batched backprojection, 24 jobs, {dt}", flush=True)
    bs = br.backprojection(gs)
    bs_ref = [op.backprojection_raw(g) for op, g in zip(ops, gs)]
    torch.cuda.synchronize()
    for i in range(len(jobs)):
        if dt == "f32":
            assert torch.equal(ys[i], ys_ref[i]), f"forward job {i}"
        else:
            a, b = ys[i].double(), ys_ref[i].double()
            d = float((a - b).norm() / b.norm())
            assert d <= 1e-3, (i, d)
        assert torch.equal(bs[i], bs_ref[i]), f"backprojection job {i}"


def test_batched_matches_oracle():
    """Batched results against the FP64 oracle: whole small jobs, sampled large ones."""
    from paper_2009_14788_amd.batched import BatchedRadon
    jobs = _jobs(12, seed=5)
    ops = _ops(jobs)
    xs = _images(jobs)
    br = BatchedRadon(ops)
    ys = br.forward(xs)
    gs = [torch.from_numpy(inputs.randn((1,) + op.sinogram_shape, 60 + i)).cuda() for i, op in enumerate(ops)]
    bs = br.backprojection(gs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    worst_f = worst_b = 0.0
    for i, j in enumerate(jobs):
        og = Case("parallel", j.n, j.angles(), j.det_count).oracle()
        x = xs[i].double().cpu().numpy()
        g = gs[i].double().cpu().numpy()
        idx = sample_indices(rng, 64, (1, j.n_angles, j.det_count))
        yf = ys[i].double().cpu().numpy()[idx[:, 0], idx[:, 1], idx[:, 2]]
        worst_f = max(worst_f, rel_l2(yf, oracle.forward_rays(og, x, idx)))
        pidx = sample_indices(rng, 8, (1, j.n, j.n))
        xb = bs[i].double().cpu().numpy()[pidx[:, 0], pidx[:, 1], pidx[:, 2]]
        worst_b = max(worst_b, rel_l2(xb, oracle.backproject_pixels(og, g, pidx)))
    report("batched_vs_oracle", fwd_worst_rel_l2=worst_f, bp_worst_rel_l2=worst_b)
    assert worst_f <= TOL_F32 and worst_b <= TOL_F32


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_batched_16bit_odd_and_even_sides(dt):
    """The 16-bit batched forward on tap pairs: odd image sides (pairs staged from 16-bit
    loads) and even ones (pairs from 32-bit words), groups of 1 to 4 images per lane,
    parallel and fan beam, every element against the FP64 oracle on the 16-bit-rounded
    images; the backprojection of the same jobs within the same bar."""
    from paper_2009_14788_amd.batched import BatchedRadon
    U = inputs.uniform_angles
    cases = [Case("parallel", 37, U(23), 53), Case("parallel", 64, U(40), 91),
             Case("parallel", 37, U(23), 53),
             Case("fanbeam", 46, U(30, 2 * math.pi), 70, 1.5, 200.0, 100.0)]
    batches = (3, 5, 1, 2)
    ops = [c.library() for c in cases]
    xs = [torch.from_numpy(inputs.randn((b, c.n, c.n), 90 + k)).cuda().to(TDT[dt])
          for k, (c, b) in enumerate(zip(cases, batches))]
    gs = [torch.from_numpy(inputs.randn((b,) + op.sinogram_shape, 95 + k)).cuda().to(TDT[dt])
          for k, (op, b) in enumerate(zip(ops, batches))]
    print(f"[gpu-step] batched 16-bit forward and backprojection, odd and even sides, {dt}", flush=True)
    br = BatchedRadon(ops)
    ys = br.forward(xs)
    bs = br.backprojection(gs)
    torch.cuda.synchronize()
    worst_f = worst_b = 0.0
    for k, c in enumerate(cases):
        og = c.oracle()
        yr = oracle.forward(og, xs[k].double().cpu().numpy())
        br_ = oracle.backproject(og, gs[k].double().cpu().numpy())
        worst_f = max(worst_f, rel_l2(ys[k].double().cpu().numpy(), yr))
        worst_b = max(worst_b, rel_l2(bs[k].double().cpu().numpy(), br_))
    report(f"batched_16bit_sides_{dt}", fwd_worst_rel_l2=worst_f, bp_worst_rel_l2=worst_b)
    assert worst_f <= TOL_16 and worst_b <= TOL_16, (worst_f, worst_b)


def test_batched_mixed_beams_and_batches():
    """Parallel and fan jobs with several images each in one launch equal per-job calls."""
    from paper_2009_14788_amd.batched import BatchedRadon
    from paper_2009_14788_amd.radon import Radon, RadonFanbeam
    ops = [Radon(96, inputs.uniform_angles(40), 137),
           RadonFanbeam(128, inputs.uniform_angles(64, 2 * math.pi), 300.0, 150.0, 190, 1.5),
           Radon(40, inputs.uniform_angles(17, 2.0), 60),
           RadonFanbeam(64, inputs.uniform_angles(30, 2 * math.pi), 200.0, 100.0, 100, 1.4)]
    xs = [torch.from_numpy(inputs.randn((b, op.resolution, op.resolution), 70 + k)).cuda()
          for k, (op, b) in enumerate(zip(ops, (3, 9, 1, 33)))]
    br = BatchedRadon(ops)
    ys = br.forward(xs, scales=[1.0, 0.5, 2.0, 1.0])
    bs = br.backprojection(ys)
    for k, op in enumerate(ops):
        s = [1.0, 0.5, 2.0, 1.0][k]
        assert torch.equal(ys[k], op.forward_raw(xs[k], s))
        assert torch.equal(bs[k], op.backprojection_raw(ys[k]))


def test_batched_graph_replay():
    """Capture batched forward + backprojection into a graph; every replay (with eager
    work, new input data and synchronisations in between) equals the eager result."""
    from paper_2009_14788_amd.batched import BatchedRadon
    jobs = _jobs(16, seed=9)
    ops = _ops(jobs)
    br = BatchedRadon(ops)
    xs = _images(jobs)
    ys = [torch.empty((1,) + op.sinogram_shape, device="cuda") for op in ops]
    bs = [torch.empty((1,) + op.image_shape, device="cuda") for op in ops]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                  # eager calls build the device tables
        br.forward(xs, out=ys)
        br.backprojection(ys, out=bs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        br.forward(xs, out=ys)
        br.backprojection(ys, out=bs)
    for rep in range(4):
        with torch.no_grad():
            for k, x in enumerate(xs):             # new data in the captured input buffers
                x.copy_(torch.from_numpy(inputs.randn(tuple(x.shape), 100 * rep + k)).cuda())
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ref_y = [op.forward_raw(x) for op, x in zip(ops, xs)]
        ref_b = [op.backprojection_raw(y) for op, y in zip(ops, ref_y)]
        torch.cuda.synchronize()
        for k in range(len(ops)):
            assert torch.equal(ys[k], ref_y[k]), (rep, k)
            assert torch.equal(bs[k], ref_b[k]), (rep, k)


def test_batched_argument_errors():
    from paper_2009_14788_amd.batched import BatchedRadon
    from paper_2009_14788_amd.radon import Radon
    br = BatchedRadon([Radon(16, inputs.uniform_angles(8), 23)])
    with pytest.raises(ValueError):
        br.forward([])
    with pytest.raises(ValueError):
        br.forward([torch.zeros((1, 15, 15), device="cuda")])
    assert br.forward([torch.zeros((0, 16, 16), device="cuda")])[0].shape == (0, 8, 23)
