"""MI355X (gfx950) discretised Radon transform: ray-driven forward projection and
its exact-transpose backprojection as hand-written HIP kernels behind a C ABI
(libradon.so, declared in include/radon.h), with a thin PyTorch binding.

Importing the package is cheap; the HIP library is loaded when a projector,
solver or binding symbol is first used, and loading fails loudly if it was not
built (there is no CPU fallback).
"""
import importlib

__all__ = ["Radon", "RadonFanbeam", "RadonForward", "RadonBackprojection", "dot_f64",
           "dot_f64_batched", "autocast_dtype", "default_fan_spacing", "release_plans",
           "power_iteration", "unrolled_gd", "Landweber", "cg", "cgne", "BatchedRadon",
           "ShearletTransform", "inputs"]

_LAZY = {
    "Radon": "radon", "RadonFanbeam": "radon", "RadonForward": "radon",
    "RadonBackprojection": "radon", "dot_f64": "radon", "default_fan_spacing": "radon",
    "release_plans": "radon", "dot_f64_batched": "radon", "autocast_dtype": "radon",
    "power_iteration": "solvers", "unrolled_gd": "solvers", "Landweber": "solvers",
    "cg": "solvers", "cgne": "solvers", "BatchedRadon": "batched",
    "ShearletTransform": "shearlet",
}


def __getattr__(name):
    if name in _LAZY:
        mod = importlib.import_module(f".{_LAZY[name]}", __name__)
        return getattr(mod, name)
    if name == "inputs":
        return importlib.import_module(".inputs", __name__)
    raise AttributeError(name)
