"""Unrolled 10-step gradient descent on the 64 x 512^2 fan-beam workload (S = 1000,
E = 500, 1024 bins x 1.5, 1024 angles over [0, 2 pi)) with 16-bit storage, against
the FP64 oracle gradient descent on whole images.

x_{k+1} = x_k - alpha R^T (R x_k - y) from x_0 = 0 (alpha inside the backprojection's
scale), run on the GPU for the whole batch of 64 in BF16 or FP16 storage; the data y
of the compared images is the oracle's projection of the phantoms (FP64, then
rounded to the storage type).  Stated per iteration: the relative L2 error of x_k
against the oracle's x_k.  Also the gradient of L = ||x_10 - x_true||^2 with respect
to y, through the checkpointed unrolled loop (autograd, the transpose kernel in the
backward pass), against the oracle's adjoint recurrence.

alpha is a fixed input shared by both sides: 0.95 / ||R||^2 with ||R||^2 = 5.2e5,
rounded up from the power-iteration estimate for this geometry (5.17e5), which keeps
every iteration contracting; the oracle runs with the same number.
"""
import numpy as np
import pytest

import oracle
from oracle import solvers
from paper_2009_14788_amd import inputs
from _helpers import rel_l2, report, workload_case

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TDT = {"f16": torch.float16, "bf16": torch.bfloat16}
ALPHA = 0.95 / 5.2e5
ITERS = 10
SEL = (0, 37)
# unit roundoff of the storage type: every iterate, residual and gradient is stored
# in it, so the error of step k can reach about k units (bars below: 2k units)
UNIT = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module")
def fan_gd():
    w = inputs.WORKLOADS["fan64_512"]
    case = workload_case(w)
    og = case.oracle()
    x = inputs.phantom_batch(4, w.batch, w.n)
    xt = x[list(SEL)].astype(np.float64)
    print(f"[gpu-step] oracle projections and 10-step GD of images {SEL}", flush=True)
    y = oracle.forward(og, xt)
    fwd = lambda v: oracle.forward(og, v)
    bp = lambda r: oracle.backproject(og, r)
    iterates, grad = solvers.unrolled_gd_grad(fwd, bp, y, ALPHA, ITERS, xt)
    return case, x, y, iterates, grad


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_unrolled_gd_fan_vs_oracle(fan_gd, dt):
    from paper_2009_14788_amd.solvers import gd_step, unrolled_gd
    case, x, y_ref, it_ref, grad_ref = fan_gd
    op = case.library()
    B = x.shape[0]
    op.prepare(TDT[dt], B)
    xt = torch.from_numpy(x).cuda().to(TDT[dt])
    with torch.no_grad():
        y = op.forward_raw(xt)                   # data of the images not compared
        y[list(SEL)] = torch.from_numpy(y_ref.astype(np.float32)).cuda().to(TDT[dt])
    print(f"[gpu-step] unrolled GD {dt} batch {B}", flush=True)
    errs = []
    with torch.no_grad():
        xk = torch.zeros_like(xt)
        for k in range(ITERS):
            xk = gd_step(op, xk, y, ALPHA)
            errs.append(rel_l2(xk[list(SEL)].double().cpu().numpy(), it_ref[k]))
    report(f"fan_gd10_{dt}_iterates", **{f"k{k + 1}": e for k, e in enumerate(errs)})
    for k, e in enumerate(errs):
        assert e <= 2 * (k + 1) * UNIT[dt], (k + 1, e)
    print(f"[gpu-step] unrolled GD backward {dt}", flush=True)
    yreq = y.clone().requires_grad_(True)
    x10 = unrolled_gd(op, yreq, ALPHA, iters=ITERS, checkpoint=True)
    ((x10.float() - xt.float()) ** 2).sum().backward()
    g = yreq.grad[list(SEL)].double().cpu().numpy()
    e_g = rel_l2(g, grad_ref)
    report(f"fan_gd10_{dt}_grad_y", rel_l2=e_g, final_iterate_rel_l2=errs[-1])
    assert e_g <= 2 * (ITERS + 1) * UNIT[dt] * 4, e_g
