"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no Radon arithmetic: it only draws random ellipse phantoms,
angle sets, noise and N(0,1) arrays, and names the benchmark workloads.  Both
the oracle-based tests and the GPU library consume what it produces.

Phantoms stand in for the Shepp-Logan phantom the paper measures on (Sec. 3.1):
sums of ellipses with random centre (uniform by area in the disc of radius
0.7*N/2), semi-axes (uniform in [0.05, 0.4]*N/2), rotation (uniform in
[0, pi)) and additive intensity (uniform in [-0.3, 1.0]).  N(0,1) batches
stand in for the `torch.randn` batches of Sec. 4.1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Ellipse:
    cx: float      # centre, centred pixel coordinates (x to the right, y down the rows)
    cy: float
    a: float       # semi-axis along the rotated x axis
    b: float       # semi-axis along the rotated y axis
    phi: float     # rotation, radians
    rho: float     # additive intensity


def ellipse_params(rng: np.random.Generator, n: int, count: int) -> list[Ellipse]:
    """Draw `count` random ellipses for an n x n image."""
    half = 0.5 * n
    out = []
    for _ in range(count):
        rad = 0.7 * half * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        a = rng.uniform(0.05, 0.4) * half
        b = rng.uniform(0.05, 0.4) * half
        phi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(-0.3, 1.0)
        out.append(Ellipse(rad * math.cos(ang), rad * math.sin(ang), a, b, phi, rho))
    return out


def rasterize(ellipses: list[Ellipse], n: int, supersample: int = 1,
              dtype=np.float32) -> np.ndarray:
    """Image [n][n] of the ellipse sum; pixel (r, c) has centre
    (c - (n-1)/2, r - (n-1)/2).  supersample=1 point-samples at pixel centres;
    supersample=m averages an m x m grid of sub-pixel points (area fraction)."""
    m = int(supersample)
    off = (np.arange(m) + 0.5) / m - 0.5
    cent = np.arange(n) - 0.5 * (n - 1)
    xs = (cent[None, :, None] + off[None, None, :]).reshape(-1)   # n*m sub-columns
    ys = xs
    img = np.zeros((n * m, n * m), dtype=np.float64)
    X = xs[None, :]
    Y = ys[:, None]
    for e in ellipses:
        c, s = math.cos(e.phi), math.sin(e.phi)
        dx = X - e.cx
        dy = Y - e.cy
        xr = dx * c + dy * s
        yr = -dx * s + dy * c
        img += e.rho * ((xr / e.a) ** 2 + (yr / e.b) ** 2 <= 1.0)
    img = img.reshape(n, m, n, m).mean(axis=(1, 3))
    return img.astype(dtype)


def phantom(n: int, count: int, seed, supersample: int = 1, dtype=np.float32):
    """One seeded phantom; returns (image, ellipses)."""
    rng = np.random.default_rng(seed)
    ell = ellipse_params(rng, n, count)
    return rasterize(ell, n, supersample, dtype), ell


def phantom_batch(config: int, batch: int, n: int, count=None, dtype=np.float32) -> np.ndarray:
    """Batch of phantoms; image i of workload `config` uses seed [config, i].
    count=None draws the ellipse count uniformly from [10, 20] (seed-dependent)."""
    out = np.empty((batch, n, n), dtype=dtype)
    for i in range(batch):
        rng = np.random.default_rng([config, i])
        k = int(rng.integers(10, 21)) if count is None else int(count)
        out[i] = rasterize(ellipse_params(rng, n, k), n, 1, dtype)
    return out


def uniform_angles(count: int, arc: float = math.pi, start: float = 0.0) -> np.ndarray:
    """theta_i = start + i*arc/count, i < count (end point excluded), float64."""
    return start + np.arange(count, dtype=np.float64) * (arc / count)


def randn(shape, seed, dtype=np.float32) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def noise(shape, sigma, seed, dtype=np.float32) -> np.ndarray:
    """Gaussian noise with per-item standard deviation sigma (array over dim 0)."""
    z = np.random.default_rng(seed).standard_normal(shape)
    sig = np.asarray(sigma, dtype=np.float64).reshape((-1,) + (1,) * (len(shape) - 1))
    return (z * sig).astype(dtype)


@dataclass
class Workload:
    name: str
    beam: str                 # "parallel" | "fanbeam"
    batch: int
    n: int
    n_angles: int
    arc: float
    det_count: int
    det_spacing: float
    source_distance: float = 0.0
    det_distance: float = 0.0
    dtypes: tuple = ("f32",)
    extra: dict = field(default_factory=dict)

    def angles(self) -> np.ndarray:
        return uniform_angles(self.n_angles, self.arc)


# The five workloads: a single 64^2 image; a 16 x 256^2 batch; the 128 x 512^2,
# 720-angle differentiable reconstruction (the headline throughput case); 200
# uneven jobs; and a 64 x 512^2 fan-beam batch with 16-bit storage.
WORKLOADS = {
    "single64": Workload("single64", "parallel", 1, 64, 64, math.pi, 91, 1.0),
    "batch16_256": Workload("batch16_256", "parallel", 16, 256, 256, math.pi, 363, 1.0),
    "batch128_512": Workload("batch128_512", "parallel", 128, 512, 720, math.pi, 724, 1.0,
                             dtypes=("f32", "f16", "bf16")),
    "fan64_512": Workload("fan64_512", "fanbeam", 64, 512, 1024, 2 * math.pi, 1024, 1.5,
                          source_distance=1000.0, det_distance=500.0, dtypes=("bf16", "f16")),
}

UNEVEN_SIZES = (128, 192, 256, 384, 512)
UNEVEN_ANGLES = (30, 60, 180, 360)
UNEVEN_ARCS = (math.pi, 2.0 * math.pi / 3.0)


@dataclass
class UnevenJob:
    n: int
    n_angles: int
    arc: float
    det_count: int
    seed: tuple

    def angles(self) -> np.ndarray:
        return uniform_angles(self.n_angles, self.arc)


def uneven_jobs(count: int = 200, seed: int = 3) -> list[UnevenJob]:
    """The uneven batch: side N from UNEVEN_SIZES, angle count from UNEVEN_ANGLES,
    arc from UNEVEN_ARCS, detector count ceil(N*sqrt(2)) of spacing 1."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(count):
        n = int(rng.choice(UNEVEN_SIZES))
        a = int(rng.choice(UNEVEN_ANGLES))
        arc = float(UNEVEN_ARCS[int(rng.integers(0, 2))])
        jobs.append(UnevenJob(n, a, arc, int(math.ceil(n * math.sqrt(2.0))), (seed, i)))
    return jobs


def uneven_phantom(job: UnevenJob, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(list(job.seed))
    k = int(rng.integers(10, 21))
    return rasterize(ellipse_params(rng, job.n, k), job.n, 1, dtype)
