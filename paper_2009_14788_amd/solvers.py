"""Iterative use of the projector pair: the operator norm by power iteration and an
unrolled gradient-descent (Landweber) reconstruction that is differentiated end to
end with per-iteration activation checkpointing.

TorchRadon runs Landweber iteration x <- x - alpha R^T (R x - y) with a step size
estimated by power iteration (Sec. 4.2, the Landweber solver).  Here alpha
defaults to exactly 1 / ||R||^2, the GPU kernels do every projection, and all
inner products and norms are FP64 reductions on the GPU.
"""
from __future__ import annotations

import math

import torch
import torch.utils.checkpoint

from .radon import dot_f64


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
