"""ctypes binding of libradon.so (argument marshalling only; every step of the
transform runs in the HIP kernels).  Raises at import if the library is missing:
there is no CPU fallback."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libradon.so")

RADON_PARALLEL = 0
RADON_FANBEAM = 1
RADON_F32, RADON_F16, RADON_BF16 = 0, 1, 2
RADON_SOLVER_LANDWEBER, RADON_SOLVER_CGNE = 0, 1
FILTERS = {"ram-lak": 0, "shepp-logan": 1, "cosine": 2, "hamming": 3, "hann": 4}

STATUS = {
    0: "RADON_OK", -1: "RADON_ERR_INVALID_ARG", -2: "RADON_ERR_ALIGN",
    -3: "RADON_ERR_UNSUPPORTED", -4: "RADON_ERR_HIP", -5: "RADON_ERR_ALLOC",
    -6: "RADON_ERR_NO_DEVICE", -7: "RADON_ERR_NOT_PREPARED", -8: "RADON_ERR_SCRATCH",
}


class RadonError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} ({string(status)})")


class Geometry(ctypes.Structure):
    _fields_ = [
        ("beam", ctypes.c_int32),
        ("image_size", ctypes.c_int32),
        ("n_angles", ctypes.c_int32),
        ("det_count", ctypes.c_int32),
        ("angles", ctypes.POINTER(ctypes.c_double)),
        ("det_spacing", ctypes.c_double),
        ("source_distance", ctypes.c_double),
        ("det_distance", ctypes.c_double),
        ("step", ctypes.c_double),
    ]


class Job(ctypes.Structure):
    _fields_ = [
        ("geometry", ctypes.POINTER(Geometry)),
        ("input", ctypes.c_void_p),
        ("output", ctypes.c_void_p),
        ("batch", ctypes.c_int32),
        ("scale", ctypes.c_float),
    ]


class Shearlet(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("n_scales", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("alphas", ctypes.POINTER(ctypes.c_double)),
    ]


def _load():
    # PyTorch ships its own HIP runtime (same soname, libamdhip64.so.7).  Loading torch
    # first makes libradon.so bind to that runtime, so that the library and torch share
    # one HIP runtime, one device context and the same streams.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(or python paper_2009_14788_amd/build.py); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    G = ctypes.POINTER(Geometry)
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    sig = {
        "radon_validate": ([G], ctypes.c_int),
        "radon_prepare": ([G, i32, i32], ctypes.c_int),
        "radon_forward": ([G, vp, vp, i32, i32, f32, vp], ctypes.c_int),
        "radon_backproject": ([G, vp, vp, i32, i32, f32, vp], ctypes.c_int),
        "radon_forward_batched": ([ctypes.POINTER(Job), i32, i32, vp], ctypes.c_int),
        "radon_backproject_batched": ([ctypes.POINTER(Job), i32, i32, vp], ctypes.c_int),
        "radon_filter_sinogram": ([G, vp, vp, i32, i32, i32, vp], ctypes.c_int),
        "radon_dot_f64": ([vp, vp, ctypes.c_int64, i32, vp, vp], ctypes.c_int),
        "radon_dot_f64_batched": ([vp, vp, ctypes.c_int64, i32, i32, vp, vp], ctypes.c_int),
        "radon_dot_f64_batched_noalloc": ([vp, vp, ctypes.c_int64, i32, i32, vp, vp], ctypes.c_int),
        "radon_axpy_ratio": ([vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int64, i32, i32, vp],
                             ctypes.c_int),
        "radon_solver_workspace_bytes": ([G, i32, i32, i32], ctypes.c_int64),
        "radon_landweber": ([G, vp, vp, i32, ctypes.c_double, i32, i32, vp, ctypes.c_int64, vp],
                            ctypes.c_int),
        "radon_cgne": ([G, vp, vp, i32, i32, i32, vp, ctypes.c_int64, vp], ctypes.c_int),
        "radon_measure_peaks": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                                ctypes.c_int),
        "radon_release_plans": ([], ctypes.c_int),
        "radon_plan_info": ([G, i32, i32, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "radon_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "radon_shearlet_channels": ([ctypes.POINTER(Shearlet)], ctypes.c_int),
        "radon_shearlet_scales": ([ctypes.POINTER(Shearlet), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "radon_shearlet_prepare": ([ctypes.POINTER(Shearlet), i32], ctypes.c_int),
        "radon_shearlet_forward": ([ctypes.POINTER(Shearlet), vp, vp, i32, i32, vp], ctypes.c_int),
        "radon_shearlet_adjoint": ([ctypes.POINTER(Shearlet), vp, vp, i32, i32, vp], ctypes.c_int),
        "radon_version": ([], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def string(status: int) -> str:
    return lib.radon_status_string(int(status)).decode()


def check(fn: str, status: int) -> None:
    if status != 0:
        raise RadonError(fn, status)
