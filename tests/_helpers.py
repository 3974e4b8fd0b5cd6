"""Shared test helpers: error measures and oracle/library geometry pairs built
from the same plain parameters (the two sides share no code)."""
import math
import sys

import numpy as np

import oracle


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def max_rel(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    m = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (m if m > 0 else 1.0))


def report(tag, **vals):
    """One greppable line per parity result (the error against the oracle)."""
    items = " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in vals.items())
    print(f"[parity] {tag} {items}", flush=True)
    sys.stdout.flush()


class Case:
    """A geometry described once, instantiated for the oracle and for the library."""

    def __init__(self, beam, n, angles, det_count, det_spacing=1.0, source_distance=0.0,
                 det_distance=0.0, step=1.0):
        self.beam = beam
        self.n = n
        self.angles = np.asarray(angles, dtype=np.float64)
        self.det_count = det_count
        self.det_spacing = det_spacing
        self.source_distance = source_distance
        self.det_distance = det_distance
        self.step = step

    def oracle(self):
        return oracle.Geometry(self.n, self.angles, self.det_count, self.det_spacing,
                               beam=oracle.FANBEAM if self.beam == "fanbeam" else oracle.PARALLEL,
                               source_distance=self.source_distance,
                               det_distance=self.det_distance, step=self.step)

    def library(self):
        from paper_2009_14788_amd.radon import Radon, RadonFanbeam
        if self.beam == "fanbeam":
            return RadonFanbeam(self.n, self.angles, self.source_distance, self.det_distance,
                                self.det_count, self.det_spacing, self.step)
        return Radon(self.n, self.angles, self.det_count, self.det_spacing, self.step)

    def __repr__(self):
        return (f"Case({self.beam}, N={self.n}, A={self.angles.size}, D={self.det_count}, "
                f"sp={self.det_spacing}, S={self.source_distance}, E={self.det_distance}, "
                f"step={self.step})")


def workload_case(w):
    return Case(w.beam, w.n, w.angles(), w.det_count, w.det_spacing, w.source_distance,
                w.det_distance)


def sample_indices(rng, count, dims):
    return np.stack([rng.integers(0, d, size=count) for d in dims], axis=1).astype(np.int64)


# FP32 parity bar (relative L2 against the FP64 oracle) and the 16-bit storage bar.
TOL_F32 = 1e-5
TOL_16 = 5e-3
