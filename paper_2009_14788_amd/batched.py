"""Uneven batches: several projectors (different image sizes, angle sets, beams) whose
forward projections or backprojections run as ONE persistent kernel launch.

The library builds the job/work tables the first time it sees a job list (by
content: projectors, buffers, batch sizes, scales) and only launches afterwards,
so a call can be captured into a CUDA/HIP graph once it has run eagerly with the
same buffers: pass preallocated outputs with `out=` for that.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .radon import _check_tensor, _stream_ptr, dtype_code


class BatchedRadon:
    def __init__(self, ops):
        self.ops = list(ops)

    def _run(self, fn_name, inputs, in_shapes, out_shapes, scales, out):
        n = len(self.ops)
        if len(inputs) != n:
            raise ValueError(f"expected {n} inputs, got {len(inputs)}")
        if n == 0:
            return []
        dtype = inputs[0].dtype
        code = dtype_code(dtype)
        dev = inputs[0].device
        scales = [1.0] * n if scales is None else [float(s) for s in scales]
        srcs, outs = [], []
        jobs = (_lib.Job * n)()
        for i, (op, t) in enumerate(zip(self.ops, inputs)):
            _check_tensor(t, f"input {i}")
            if t.dtype != dtype or t.device != dev:
                raise ValueError("all inputs must share dtype and device")
            if tuple(t.shape[-2:]) != tuple(in_shapes[i]):
                raise ValueError(f"input {i}: expected trailing shape {tuple(in_shapes[i])}")
            lead = tuple(t.shape[:-2])
            batch = int(np.prod(lead)) if lead else 1
            src = t.contiguous()
            if src.data_ptr() % 16:
                src = src.clone()
            if out is not None:
                o = out[i]
                if (tuple(o.shape) != lead + tuple(out_shapes[i]) or o.dtype != dtype
                        or not o.is_contiguous() or o.data_ptr() % 16):
                    raise ValueError(f"out[{i}] must be a contiguous, 16-byte aligned "
                                     f"{lead + tuple(out_shapes[i])} tensor of {dtype}")
            else:
                o = torch.empty(lead + tuple(out_shapes[i]), dtype=dtype, device=dev)
            srcs.append(src)
            outs.append(o)
            jobs[i].geometry = ctypes.pointer(op.geometry)
            jobs[i].input = src.data_ptr() if batch else None
            jobs[i].output = o.data_ptr() if batch else None
            jobs[i].batch = batch
            jobs[i].scale = scales[i]
        with torch.cuda.device(dev):
            rc = getattr(_lib.lib, fn_name)(jobs, n, code, _stream_ptr(dev))
        _lib.check(fn_name, rc)
        return outs

    def forward(self, xs, scales=None, out=None):
        """Sinograms scale_i * R_i x_i for every job i, in one launch."""
        return self._run("radon_forward_batched", xs, [op.image_shape for op in self.ops],
                         [op.sinogram_shape for op in self.ops], scales, out)

    def backprojection(self, ys, scales=None, out=None):
        """Backprojections scale_i * R_i^T y_i for every job i, in one launch."""
        return self._run("radon_backproject_batched", ys, [op.sinogram_shape for op in self.ops],
                         [op.image_shape for op in self.ops], scales, out)
