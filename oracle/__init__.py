"""FP64 CPU oracle of the discretised Radon transform (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and this package imports
nothing from it.  The arithmetic lives in ``radon_oracle.c``; this module only
marshals NumPy float64 arrays through ctypes.

Operator (conventions stated in the C file's header; the paper, TorchRadon,
arXiv 2009.14788, fixes the geometry in Sec. 3.1.1-3.1.2 and the use of the
backprojection as the adjoint in Sec. 4.3):
    forward        y = scale * R x,   R[(a,d),(r,c)] = dt * sum_k L(P_kx-X_c) L(P_ky-Y_r)
    backprojection x = scale * R^T y
All functions are pinned by tests/test_oracle_pins.py (closed forms,
invariants, brute force and a hand-computed fixture); none is "parity unpinned".
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

PARALLEL = 0
FANBEAM = 1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.path.join(_HERE, "liboracle.so")
    src = os.path.join(_HERE, "radon_oracle.c")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        _build.build()
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    geom = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.oracle_forward.argtypes = geom + [dp, ctypes.c_int, ctypes.c_double, dp]
    lib.oracle_forward.restype = ctypes.c_int
    lib.oracle_backproject.argtypes = geom + [dp, ctypes.c_int, ctypes.c_double, dp]
    lib.oracle_backproject.restype = ctypes.c_int
    lib.oracle_matrix_entry.argtypes = geom + [ctypes.c_int] * 4
    lib.oracle_matrix_entry.restype = ctypes.c_double
    lib.oracle_dense_matrix.argtypes = geom + [dp]
    lib.oracle_dense_matrix.restype = ctypes.c_int
    lib.oracle_forward_rays.argtypes = geom + [dp, ctypes.c_double, ctypes.c_long, i64p, dp]
    lib.oracle_forward_rays.restype = ctypes.c_int
    lib.oracle_backproject_pixels.argtypes = geom + [dp, ctypes.c_double, ctypes.c_long, i64p, dp]
    lib.oracle_backproject_pixels.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


class Geometry:
    """Plain geometry record for the oracle (its own; not the library's)."""

    def __init__(self, n, angles, det_count, det_spacing=1.0, beam=PARALLEL,
                 source_distance=0.0, det_distance=0.0, step=1.0):
        self.n = int(n)
        self.angles = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).ravel())
        self.det_count = int(det_count)
        self.det_spacing = float(det_spacing)
        self.beam = int(beam)
        self.source_distance = float(source_distance)
        self.det_distance = float(det_distance)
        self.step = float(step)

    @property
    def n_angles(self):
        return int(self.angles.size)

    def _args(self):
        return (self.beam, self.n, self.n_angles, _dptr(self.angles), self.det_count,
                self.det_spacing, self.source_distance, self.det_distance, self.step)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def forward(g: Geometry, x, scale=1.0):
    """y[B][A][D] = scale * R x for x[B][N][N] (or [N][N])."""
    lib = _load()
    x = _f64(x)
    squeeze = x.ndim == 2
    xb = x.reshape(-1, g.n, g.n)
    y = np.empty((xb.shape[0], g.n_angles, g.det_count), dtype=np.float64)
    rc = lib.oracle_forward(*g._args(), _dptr(xb), xb.shape[0], float(scale), _dptr(y))
    if rc != 0:
        raise ValueError("oracle_forward: invalid geometry")
    return y[0] if squeeze else y


def backproject(g: Geometry, y, scale=1.0):
    """x[B][N][N] = scale * R^T y for y[B][A][D] (or [A][D]); scatter form."""
    lib = _load()
    y = _f64(y)
    squeeze = y.ndim == 2
    yb = y.reshape(-1, g.n_angles, g.det_count)
    x = np.empty((yb.shape[0], g.n, g.n), dtype=np.float64)
    rc = lib.oracle_backproject(*g._args(), _dptr(yb), yb.shape[0], float(scale), _dptr(x))
    if rc == -2:
        raise MemoryError("oracle_backproject: accumulators could not be allocated")
    if rc != 0:
        raise ValueError("oracle_backproject: invalid geometry")
    return x[0] if squeeze else x


def matrix_entry(g: Geometry, a, d, r, c):
    return float(_load().oracle_matrix_entry(*g._args(), int(a), int(d), int(r), int(c)))


def dense_matrix(g: Geometry):
    """R as a dense [A*D][N*N] array (small N only)."""
    lib = _load()
    m = np.empty((g.n_angles * g.det_count, g.n * g.n), dtype=np.float64)
    if lib.oracle_dense_matrix(*g._args(), _dptr(m)) != 0:
        raise ValueError("oracle_dense_matrix: invalid geometry")
    return m


def forward_rays(g: Geometry, x, idx, scale=1.0):
    """Forward outputs at idx = int array [n][3] of (b, a, d)."""
    lib = _load()
    xb = _f64(x).reshape(-1, g.n, g.n)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1, 3))
    out = np.empty(idx.shape[0], dtype=np.float64)
    rc = lib.oracle_forward_rays(*g._args(), _dptr(xb), float(scale), idx.shape[0],
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(out))
    if rc != 0:
        raise ValueError("oracle_forward_rays: invalid geometry")
    return out


def backproject_pixels(g: Geometry, y, idx, scale=1.0):
    """Backprojection outputs at idx = int array [n][3] of (b, r, c)."""
    lib = _load()
    yb = _f64(y).reshape(-1, g.n_angles, g.det_count)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1, 3))
    out = np.empty(idx.shape[0], dtype=np.float64)
    rc = lib.oracle_backproject_pixels(*g._args(), _dptr(yb), float(scale), idx.shape[0],
                                       idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(out))
    if rc != 0:
        raise ValueError("oracle_backproject_pixels: invalid geometry")
    return out


def num_threads():
    return int(_load().oracle_num_threads())


def set_num_threads(n):
    """Threads the oracle's OpenMP loops use from now on (for timing only)."""
    _load().oracle_set_num_threads(int(n))
