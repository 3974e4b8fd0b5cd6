"""Iterative use of the projector pair: the operator norm by power iteration, an
unrolled gradient-descent (Landweber) reconstruction that is differentiated end to
end with per-iteration activation checkpointing, and the solvers of TorchRadon
Sec. 4.2-4.3: Landweber iteration, conjugate gradient for an SPD operator given as a
closure, and CG on the normal equations (CGNE).

TorchRadon runs Landweber iteration x <- x - alpha R^T (R x - y) with a step size
estimated by power iteration (Sec. 4.2, the Landweber solver).  Here alpha
defaults to exactly 1 / ||R||^2, the GPU kernels do every projection, and all
inner products and norms are FP64 reductions on the GPU; the CG scalars stay on the
device, so no iteration waits on the host.
"""
from __future__ import annotations

import math

import torch
import torch.utils.checkpoint

from . import _lib
from .radon import _aligned, axpy_ratio_, dot_f64, dot_f64_batched, dtype_code


def power_iteration(op, iters: int = 200, tol: float = 1e-7, seed: int = 0,
                    dtype=torch.float32, device=None) -> float:
    """Largest eigenvalue of R^T R (that is ||R||_2^2) for projector `op`, by power
    iteration from a seeded N(0,1) image; stops when the Rayleigh quotient changes
    by less than tol (relative) or after `iters` iterations."""
    dev = torch.device("cuda") if device is None else torch.device(device)
    gen = torch.Generator().manual_seed(int(seed))
    x = torch.randn(op.image_shape, generator=gen, dtype=torch.float32).to(dev, dtype)
    x = x / math.sqrt(dot_f64(x, x).item())
    lam_prev = None
    lam = 0.0
    for _ in range(int(iters)):
        z = op.backprojection_raw(op.forward_raw(x))
        lam = dot_f64(x, z).item()                     # Rayleigh quotient, |x| = 1
        x = z / math.sqrt(dot_f64(z, z).item())
        if lam_prev is not None and abs(lam - lam_prev) <= tol * abs(lam):
            break
        lam_prev = lam
    return lam


def gd_step(op, x: torch.Tensor, y: torch.Tensor, alpha: float) -> torch.Tensor:
    """One Landweber / gradient step on 0.5 ||R x - y||^2:  x - alpha R^T (R x - y).
    alpha is applied inside the backprojection kernel (its scale argument), so 16-bit
    storage never holds the unscaled R^T r (which can exceed the FP16 range)."""
    return x - op.backprojection(op.forward(x) - y, scale=alpha)


def unrolled_gd(op, y: torch.Tensor, alpha: float, iters: int = 10, x0=None,
                checkpoint: bool = True) -> torch.Tensor:
    """x_k after `iters` gradient steps from x0 (default 0).  Differentiable in y (and
    x0); with checkpoint=True each iteration's activations are recomputed in the
    backward pass instead of being kept (one image-sized tensor kept per step)."""
    lead = y.shape[:-2]
    x = torch.zeros(tuple(lead) + op.image_shape, dtype=y.dtype, device=y.device) if x0 is None else x0
    for _ in range(int(iters)):
        if checkpoint:
            x = torch.utils.checkpoint.checkpoint(gd_step, op, x, y, alpha, use_reentrant=False)
        else:
            x = gd_step(op, x, y, alpha)
    return x


def _systems(t: torch.Tensor) -> int:
    """Independent systems of a (..., H, W) tensor: the product of its leading dims."""
    lead = t.shape[:-2]
    return int(math.prod(lead)) if len(lead) else 1


def _solver_call(fn_name, op, y, x, solver, *args):
    """Queue libradon's solver loop `fn_name` in place on x (batch = leading dims)."""
    if tuple(x.shape[-2:]) != tuple(op.image_shape):
        raise ValueError(f"guess must end in {tuple(op.image_shape)}, got {tuple(x.shape)}")
    if tuple(y.shape[-2:]) != tuple(op.sinogram_shape) or y.shape[:-2] != x.shape[:-2]:
        raise ValueError(f"sinogram shape {tuple(y.shape)} does not match guess {tuple(x.shape)}")
    if y.dtype != x.dtype:
        raise ValueError("sinogram and guess must have the same dtype")
    code = dtype_code(x.dtype)
    batch = _systems(x)
    op.prepare(x.dtype, batch, x.device)          # tuned launch shapes for this batch
    nbytes = _lib.lib.radon_solver_workspace_bytes(op.geometry, solver, batch, code)
    if nbytes < 0:
        _lib.check("radon_solver_workspace_bytes", int(nbytes))
    ws = torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=x.device)
    with torch.cuda.device(x.device):
        rc = getattr(_lib.lib, fn_name)(op.geometry, y.data_ptr(), x.data_ptr(), batch, *args, code,
                                        ws.data_ptr(), int(nbytes),
                                        torch.cuda.current_stream(x.device).cuda_stream)
    _lib.check(fn_name, rc)
    return x


def _start(guess: torch.Tensor, sino: torch.Tensor):
    if guess.device.type != "cuda" or sino.device.type != "cuda":
        raise ValueError("guess and sinogram must be on a GPU; there is no CPU path")
    x = guess.detach().contiguous().clone()
    y = sino.detach().contiguous()
    return x, (y.clone() if y.data_ptr() % 16 else y)


class Landweber:
    """Landweber iteration x <- x - alpha R^T (R x - y) for projector `op` (TorchRadon
    Sec. 4.2); each leading index of the guess is its own image.  The loop runs in
    libradon (radon_landweber): alpha is applied inside the backprojection kernel."""

    def __init__(self, op):
        self.op = op

    def estimate_alpha(self, img_size=None, device=None, n_iter: int = 200, seed: int = 0) -> float:
        """1 / ||R||^2 by power iteration (the image size is the projector's own; the
        paper's example multiplies the estimate by 0.95 for safety)."""
        return 1.0 / power_iteration(self.op, iters=n_iter, seed=seed, device=device)

    def run(self, guess: torch.Tensor, sino: torch.Tensor, alpha: float,
            iterations: int = 100) -> torch.Tensor:
        """x after `iterations` steps from `guess` (guess is not modified)."""
        x, y = _start(guess, sino)
        return _solver_call("radon_landweber", self.op, y, x, _lib.RADON_SOLVER_LANDWEBER,
                            float(alpha), int(iterations))


def cgne(op, x0: torch.Tensor, y: torch.Tensor, max_iter: int = 500) -> torch.Tensor:
    """Conjugate gradient on the normal equations R^T R x = R^T y (TorchRadon Sec. 4.2),
    `max_iter` steps from x0, every leading index its own system.  The loop runs in
    libradon (radon_cgne) in the form that keeps the residual in data space and never
    forms R^T R; FP64 inner products; float32 only."""
    x, yy = _start(x0, y)
    return _solver_call("radon_cgne", op, yy, x, _lib.RADON_SOLVER_CGNE, int(max_iter))


def cg(forward_fn, x0: torch.Tensor, y: torch.Tensor, max_iter: int = 50,
       batched: bool = True) -> torch.Tensor:
    """Conjugate gradient for A x = y with A symmetric positive definite, given as the
    closure forward_fn (TorchRadon Sec. 4.3 uses it inside ADMM).  With batched=True
    every leading index of x0 (all dims but the last two) is its own system, which
    requires A to act on each separately; batched=False treats the whole tensor as one
    system.  FP64 inner products (radon_dot_f64_batched) and updates
    (radon_axpy_ratio) with the coefficients kept on the device."""
    x, b = _start(x0, y)
    if b.shape != x.shape or b.dtype != x.dtype:
        raise ValueError("x0 and y must have the same shape and dtype")
    k = _systems(x) if batched else 1
    r = forward_fn(x).to(x.dtype).contiguous().clone()      # own storage: updated in place
    axpy_ratio_(r, b, r, c0=-1.0, systems=k)                 # r = y - A x
    p = r.clone()
    rr = dot_f64_batched(r, r, k)
    for _ in range(int(max_iter)):
        ap = _aligned(forward_fn(p).to(x.dtype))
        pap = dot_f64_batched(p, ap, k)
        axpy_ratio_(x, x, p, rr, pap, 1.0, k)                # x += a p
        axpy_ratio_(r, r, ap, rr, pap, -1.0, k)              # r -= a A p
        rr_new = dot_f64_batched(r, r, k)
        axpy_ratio_(p, r, p, rr_new, rr, 1.0, k)             # p = r + b p
        rr = rr_new
    return x
