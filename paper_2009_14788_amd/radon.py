"""PyTorch-facing API: Radon (parallel beam) and RadonFanbeam (flat-detector fan
beam), mirroring TorchRadon's constructors and methods (Sec. 3.1.1, 3.1.2, 4.1),
with autograd through the hand-written transpose kernels (Sec. 2, "Differentiability").

Torch provides device memory and streams only; every projection runs in
libradon.so.  Tensors must be CUDA (ROCm) tensors of float32, float16 or bfloat16.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib

_DTYPES = {torch.float32: _lib.RADON_F32, torch.float16: _lib.RADON_F16,
           torch.bfloat16: _lib.RADON_BF16}


def dtype_code(t: torch.dtype) -> int:
    try:
        return _DTYPES[t]
    except KeyError:
        raise TypeError(f"unsupported dtype {t}; use float32, float16 or bfloat16") from None


def autocast_dtype(t: torch.Tensor) -> torch.dtype:
    """Storage type a differentiable projection of t runs in.  Under torch.autocast on
    the GPU with a 16-bit type, an FP32 input is projected with that storage type (16-bit
    data, FP32 arithmetic: the half-precision mode of TorchRadon Sec. 3.3, usable with
    AMP as Sec. 2 states); otherwise t's own type."""
    if t.dtype == torch.float32 and torch.is_autocast_enabled("cuda"):
        dt = torch.get_autocast_dtype("cuda")
        if dt in (torch.float16, torch.bfloat16):
            return dt
    return t.dtype


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_tensor(t: torch.Tensor, what: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must be on a GPU (got {t.device}); there is no CPU path")


class _Base:
    """Common plumbing of both geometries."""

    beam = _lib.RADON_PARALLEL

    def __init__(self, resolution, angles, det_count, det_spacing, step,
                 source_distance=0.0, det_distance=0.0):
        self.resolution = int(resolution)
        self.angles = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).ravel())
        self.det_count = int(det_count)
        self.det_spacing = float(det_spacing)
        self.step = float(step)
        self.source_distance = float(source_distance)
        self.det_distance = float(det_distance)
        self._geom = _lib.Geometry(
            self.beam, self.resolution, int(self.angles.size), self.det_count,
            self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            self.det_spacing, self.source_distance, self.det_distance, self.step)
        _lib.check("radon_validate", _lib.lib.radon_validate(ctypes.byref(self._geom)))

    # ---------------------------------------------------------------- shapes
    @property
    def n_angles(self) -> int:
        return int(self.angles.size)

    @property
    def image_shape(self):
        return (self.resolution, self.resolution)

    @property
    def sinogram_shape(self):
        return (self.n_angles, self.det_count)

    @property
    def geometry(self) -> _lib.Geometry:
        return self._geom

    # ---------------------------------------------------------------- raw calls
    def _raw(self, fn_name, inp: torch.Tensor, in_shape, out_shape, scale: float) -> torch.Tensor:
        _check_tensor(inp, "input")
        if tuple(inp.shape[-2:]) != tuple(in_shape):
            raise ValueError(f"expected trailing shape {tuple(in_shape)}, got {tuple(inp.shape)}")
        code = dtype_code(inp.dtype)
        lead = inp.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        src = inp.contiguous()
        if src.data_ptr() % 16:
            src = src.clone()          # the library needs 16-byte aligned buffers
        out = torch.empty(tuple(lead) + tuple(out_shape), dtype=inp.dtype, device=inp.device)
        if batch == 0:
            return out
        with torch.cuda.device(inp.device):
            rc = getattr(_lib.lib, fn_name)(ctypes.byref(self._geom), src.data_ptr(), out.data_ptr(),
                                            batch, code, float(scale), _stream_ptr(inp.device))
        _lib.check(fn_name, rc)
        return out

    def forward_raw(self, x: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
        """scale * R x without autograd; x has shape (..., N, N)."""
        return self._raw("radon_forward", x, self.image_shape, self.sinogram_shape, scale)

    def backprojection_raw(self, y: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
        """scale * R^T y without autograd; y has shape (..., A, D)."""
        return self._raw("radon_backproject", y, self.sinogram_shape, self.image_shape, scale)

    # ---------------------------------------------------------------- autograd-aware
    def forward(self, x: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
        """Sinogram scale * R x; differentiable (the gradient is scale * R^T g, formed
        in x's own type).  Under torch.autocast an FP32 x is projected in the autocast
        16-bit type (see autocast_dtype) and its gradient still comes back in FP32."""
        return RadonForward.apply(x, self, float(scale), autocast_dtype(x))

    def backprojection(self, y: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
        """Backprojection scale * R^T y; differentiable (the gradient is scale * R g,
        formed in y's own type); autocast as for forward."""
        return RadonBackprojection.apply(y, self, float(scale), autocast_dtype(y))

    # the paper's ADMM example calls the backprojection `backward` (Sec. 4.3)
    backward = backprojection

    def filter_sinogram_raw(self, y: torch.Tensor, filter_name: str = "ram-lak") -> torch.Tensor:
        """The FBP filter without autograd (see filter_sinogram)."""
        _check_tensor(y, "input")
        if self.beam != _lib.RADON_PARALLEL:
            raise NotImplementedError("filter_sinogram: parallel beam only")
        if tuple(y.shape[-2:]) != tuple(self.sinogram_shape):
            raise ValueError(f"expected trailing shape {tuple(self.sinogram_shape)}, got {tuple(y.shape)}")
        if filter_name not in _lib.FILTERS:
            raise ValueError(f"unknown filter {filter_name!r}; one of {tuple(_lib.FILTERS)}")
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        src = y.contiguous()
        if src.data_ptr() % 16:
            src = src.clone()
        out = torch.empty_like(src)
        if batch == 0:
            return out
        with torch.cuda.device(y.device):
            rc = _lib.lib.radon_filter_sinogram(ctypes.byref(self._geom), src.data_ptr(), out.data_ptr(),
                                                batch, _lib.FILTERS[filter_name], dtype_code(y.dtype),
                                                _stream_ptr(y.device))
        _lib.check("radon_filter_sinogram", rc)
        return out

    def filter_sinogram(self, y: torch.Tensor, filter_name: str = "ram-lak") -> torch.Tensor:
        """Filter of filtered backprojection (TorchRadon Sec. 3.1.3): each projection is
        filtered in the frequency domain by the Kak & Slaney band-limited ramp (ch. 3
        eq. 61) times the window of `filter_name` ("ram-lak", "shepp-logan", "cosine",
        "hamming", "hann") and scaled by pi / A, so that
        ``backprojection(filter_sinogram(y))`` reconstructs the image when the angles
        cover [0, pi) uniformly, at any det_spacing.  Parallel beam.  Differentiable: the filter is
        symmetric, so its gradient is the same filter.  Under torch.autocast a 16-bit
        sinogram is filtered in FP32 and the result is FP32, as the paper's
        half-precision FBP filters in single precision (Sec. 3.3)."""
        if y.dtype in (torch.float16, torch.bfloat16) and torch.is_autocast_enabled("cuda"):
            y = y.float()
        return RadonFilter.apply(y, self, filter_name)

    def prepare(self, dtype=torch.float32, batch: int = 1, device=None) -> None:
        """Build the plan (tables, launch shapes) before stream capture."""
        dev = torch.device("cuda") if device is None else torch.device(device)
        with torch.cuda.device(dev):
            _lib.check("radon_prepare", _lib.lib.radon_prepare(
                ctypes.byref(self._geom), dtype_code(dtype), int(batch)))

    def plan_info(self, dtype=torch.float32, batch: int = 1):
        """Launch shapes used for this storage type and batch size, per direction:
        images per lane, angles per block, staging (1 = interleaved workspace copy,
        2 = 16-bit tap pairs), variant (1 = tiled kernel, 0 = direct kernel), and the
        forward's slab rows / the backprojection's tile side."""
        out = (ctypes.c_int32 * 10)()
        _lib.check("radon_plan_info", _lib.lib.radon_plan_info(
            ctypes.byref(self._geom), dtype_code(dtype), int(batch), out))
        keys = ("images", "angles", "staging", "variant")
        return {"forward": dict(zip(keys + ("rows",), out[0:5])),
                "backprojection": dict(zip(keys + ("tile",), out[5:10]))}


class Radon(_Base):
    """Parallel-beam projector: Radon(resolution, angles, det_count=resolution,
    det_spacing=1.0, step=1.0) as in TorchRadon Sec. 3.1.1."""

    beam = _lib.RADON_PARALLEL

    def __init__(self, resolution, angles, det_count=None, det_spacing=1.0, step=1.0):
        det_count = int(resolution) if det_count is None else int(det_count)
        super().__init__(resolution, angles, det_count, det_spacing, step)


def default_fan_spacing(resolution, source_distance, det_distance, det_count) -> float:
    """Smallest detector spacing whose fan covers the image (Sec. 3.1.2):
    (S + E) / S * N / D; 2.0 for N = 512, S = E = 512, D = 512."""
    return (source_distance + det_distance) / source_distance * resolution / det_count


class RadonFanbeam(_Base):
    """Flat-detector fan-beam projector: RadonFanbeam(resolution, angles,
    source_distance, det_distance=source_distance, det_count=resolution,
    det_spacing=<covering spacing>, step=1.0) as in TorchRadon Sec. 3.1.2."""

    beam = _lib.RADON_FANBEAM

    def __init__(self, resolution, angles, source_distance, det_distance=None, det_count=None,
                 det_spacing=None, step=1.0):
        S = float(source_distance)
        E = S if det_distance is None else float(det_distance)
        D = int(resolution) if det_count is None else int(det_count)
        sp = default_fan_spacing(resolution, S, E, D) if det_spacing is None else float(det_spacing)
        super().__init__(resolution, angles, D, sp, step, S, E)


def _grad_in(g: torch.Tensor, dtype: torch.dtype) -> torch.Tensor:
    g = g.contiguous()
    return g if g.dtype == dtype else g.to(dtype)


class RadonForward(torch.autograd.Function):
    """y = scale * R x stored as `dtype`; backward applies the hand-written transpose
    kernel in x's own type (so a 16-bit forward of an FP32 input has an FP32 gradient,
    which cannot overflow the 16-bit range)."""

    @staticmethod
    def forward(ctx, x, op, scale, dtype):
        ctx.op = op
        ctx.scale = scale
        ctx.in_dtype = x.dtype
        return op.forward_raw(x if x.dtype == dtype else x.to(dtype), scale)

    @staticmethod
    def backward(ctx, g):
        return ctx.op.backprojection_raw(_grad_in(g, ctx.in_dtype), ctx.scale), None, None, None


class RadonBackprojection(torch.autograd.Function):
    """x = scale * R^T y stored as `dtype`; backward applies the forward kernel in y's
    own type."""

    @staticmethod
    def forward(ctx, y, op, scale, dtype):
        ctx.op = op
        ctx.scale = scale
        ctx.in_dtype = y.dtype
        return op.backprojection_raw(y if y.dtype == dtype else y.to(dtype), scale)

    @staticmethod
    def backward(ctx, g):
        return ctx.op.forward_raw(_grad_in(g, ctx.in_dtype), ctx.scale), None, None, None


class RadonFilter(torch.autograd.Function):
    """FBP filter; its matrix is symmetric (the kernel is even), so backward filters
    the gradient with the same kernel."""

    @staticmethod
    def forward(ctx, y, op, name):
        ctx.op = op
        ctx.name = name
        return op.filter_sinogram_raw(y, name)

    @staticmethod
    def backward(ctx, g):
        return ctx.op.filter_sinogram_raw(g.contiguous(), ctx.name), None, None


def dot_f64(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """sum(a*b) accumulated in FP64 on the GPU (deterministic); returns a 0-d
    float64 tensor on a's device."""
    _check_tensor(a, "a")
    _check_tensor(b, "b")
    if a.shape != b.shape or a.dtype != b.dtype:
        raise ValueError("a and b must have the same shape and dtype")
    a = a.contiguous()
    b = b.contiguous()
    a = a.clone() if a.data_ptr() % 16 else a
    b = b.clone() if b.data_ptr() % 16 else b
    out = torch.empty((), dtype=torch.float64, device=a.device)
    with torch.cuda.device(a.device):
        rc = _lib.lib.radon_dot_f64(a.data_ptr(), b.data_ptr(), a.numel(), dtype_code(a.dtype),
                                    out.data_ptr(), _stream_ptr(a.device))
    _lib.check("radon_dot_f64", rc)
    return out


def _aligned(t: torch.Tensor) -> torch.Tensor:
    t = t.contiguous()
    return t.clone() if t.data_ptr() % 16 else t


def dot_f64_batched(a: torch.Tensor, b: torch.Tensor, systems: int) -> torch.Tensor:
    """Per-system FP64 inner products: the tensors are `systems` equal parts stored one
    after another; returns a float64 tensor [systems] on a's device (deterministic)."""
    _check_tensor(a, "a")
    _check_tensor(b, "b")
    if a.shape != b.shape or a.dtype != b.dtype:
        raise ValueError("a and b must have the same shape and dtype")
    systems = int(systems)
    if systems < 1 or a.numel() % systems:
        raise ValueError(f"{a.numel()} elements do not split into {systems} systems")
    a, b = _aligned(a), _aligned(b)
    out = torch.empty(systems, dtype=torch.float64, device=a.device)
    with torch.cuda.device(a.device):
        rc = _lib.lib.radon_dot_f64_batched(a.data_ptr(), b.data_ptr(), a.numel() // systems,
                                            systems, dtype_code(a.dtype), out.data_ptr(),
                                            _stream_ptr(a.device))
    _lib.check("radon_dot_f64_batched", rc)
    return out


def axpy_ratio_(out: torch.Tensor, u: torch.Tensor, v: torch.Tensor, num=None, den=None,
                c0: float = 1.0, systems: int = 1) -> torch.Tensor:
    """In place: out_k = u_k + c_k v_k for each of `systems` equal parts, with
    c_k = c0 * num[k] / den[k] (float64 device tensors or None; c_k = 0 where
    den[k] == 0).  out may be u or v; all three contiguous, same shape and dtype."""
    for t, w in ((out, "out"), (u, "u"), (v, "v")):
        _check_tensor(t, w)
        if t.shape != out.shape or t.dtype != out.dtype:
            raise ValueError("out, u and v must have the same shape and dtype")
        if not t.is_contiguous() or t.data_ptr() % 16:
            raise ValueError(f"{w} must be contiguous and 16-byte aligned")
    systems = int(systems)
    if systems < 1 or out.numel() % systems:
        raise ValueError(f"{out.numel()} elements do not split into {systems} systems")
    ptrs = []
    for c in (num, den):
        if c is None:
            ptrs.append(None)
            continue
        if c.dtype != torch.float64 or c.numel() != systems or c.device != out.device:
            raise ValueError("num and den must be float64 tensors with one entry per system")
        ptrs.append(c.contiguous().data_ptr())
    with torch.cuda.device(out.device):
        rc = _lib.lib.radon_axpy_ratio(u.data_ptr(), v.data_ptr(), out.data_ptr(), ptrs[0], ptrs[1],
                                       float(c0), out.numel() // systems, systems,
                                       dtype_code(out.dtype), _stream_ptr(out.device))
    _lib.check("radon_axpy_ratio", rc)
    return out


def release_plans() -> None:
    _lib.check("radon_release_plans", _lib.lib.radon_release_plans())
