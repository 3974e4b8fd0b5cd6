"""Alpha-shearlet transform on the GPU (TorchRadon Sec. 2.1 and 3.2):
ShearletTransform(width, height, alphas) with `forward` (coefficients) and `backward`
(the adjoint, which inverts the Parseval frame), differentiable, for batches.

The Fourier filters are built once by libradon.so; every transform is the library's
FFT kernels (radon_shearlet_forward / radon_shearlet_adjoint).  Torch provides
device memory and streams only.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .radon import _check_tensor, _stream_ptr, dtype_code


class ShearletTransform:
    """Real-valued alpha-shearlets for width x height images (powers of two, 16..4096),
    one alpha per scale, e.g. ShearletTransform(512, 512, [0.5] * 5) (59 channels).

    forward(x): x[..., H, W] -> coefficients [..., M, H, W]
    backward(c): coefficients [..., M, H, W] -> images [..., H, W] (the adjoint; since
    the frame is Parseval, backward(forward(x)) = x)
    scales: tensor [M] with the scale of each channel (0 for the low-pass, j + 1 for
    scale j), as the paper's regularised reconstruction uses it to weigh channels."""

    def __init__(self, width: int, height: int, alphas):
        self.width = int(width)
        self.height = int(height)
        self.alphas = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).ravel())
        self._s = _lib.Shearlet(self.width, self.height, int(self.alphas.size), 0,
                                self.alphas.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        m = _lib.lib.radon_shearlet_channels(ctypes.byref(self._s))
        if m < 0:
            _lib.check("radon_shearlet_channels", m)
        self.channels = int(m)
        sc = (ctypes.c_int32 * self.channels)()
        _lib.check("radon_shearlet_scales", _lib.lib.radon_shearlet_scales(ctypes.byref(self._s), sc))
        self.scales = torch.tensor(list(sc), dtype=torch.int64)

    def prepare(self, batch: int = 1, device=None) -> None:
        """Build the filters and the null stream's workspace for `batch` images."""
        dev = torch.device("cuda") if device is None else torch.device(device)
        with torch.cuda.device(dev):
            _lib.check("radon_shearlet_prepare",
                       _lib.lib.radon_shearlet_prepare(ctypes.byref(self._s), int(batch)))

    def _run(self, fn, t, in_tail, out_tail):
        _check_tensor(t, "input")
        if tuple(t.shape[-len(in_tail):]) != in_tail:
            raise ValueError(f"expected trailing shape {in_tail}, got {tuple(t.shape)}")
        lead = tuple(t.shape[:-len(in_tail)])
        batch = int(np.prod(lead)) if lead else 1
        src = t.contiguous()
        if src.data_ptr() % 16:
            src = src.clone()
        out = torch.empty(lead + out_tail, dtype=t.dtype, device=t.device)
        if batch:
            with torch.cuda.device(t.device):
                rc = getattr(_lib.lib, fn)(ctypes.byref(self._s), src.data_ptr(), out.data_ptr(), batch,
                                           dtype_code(t.dtype), _stream_ptr(t.device))
            _lib.check(fn, rc)
        return out

    def forward_raw(self, x: torch.Tensor) -> torch.Tensor:
        return self._run("radon_shearlet_forward", x, (self.height, self.width),
                         (self.channels, self.height, self.width))

    def backward_raw(self, c: torch.Tensor) -> torch.Tensor:
        return self._run("radon_shearlet_adjoint", c, (self.channels, self.height, self.width),
                         (self.height, self.width))

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """Shearlet coefficients of x (differentiable: the gradient is the adjoint)."""
        return _ShearletForward.apply(x, self)

    def backward(self, c: torch.Tensor) -> torch.Tensor:
        """Adjoint transform of c (differentiable: the gradient is the forward)."""
        return _ShearletAdjoint.apply(c, self)


class _ShearletForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, sh):
        ctx.sh = sh
        return sh.forward_raw(x)

    @staticmethod
    def backward(ctx, g):
        return ctx.sh.backward_raw(g), None


class _ShearletAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, sh):
        ctx.sh = sh
        return sh.backward_raw(c)

    @staticmethod
    def backward(ctx, g):
        return ctx.sh.forward_raw(g), None
