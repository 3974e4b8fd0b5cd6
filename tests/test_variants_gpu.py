"""Every launch-shape variant the autotuner can choose gives the same results: forward
with 4/8/16 images per lane and either slab staging (bitwise identical), and
backprojection with 16/32 images per lane and 4/8-angle LDS blocks (identical up to
the grouping of the FP32 partial sums).  Also checks that autotuning runs and keeps
results within the parity bar."""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2009_14788_amd import inputs
from _helpers import Case, TOL_F32, rel_l2, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2009_14788_amd import inputs
from paper_2009_14788_amd.radon import Radon, RadonFanbeam
import math
out = {}
for name, op, dt in [("par", Radon(96, inputs.uniform_angles(60), 137), torch.float32),
                     ("par16", Radon(96, inputs.uniform_angles(60), 137), torch.float16),
                     ("fan", RadonFanbeam(96, inputs.uniform_angles(60, 2 * math.pi), 250.0, 120.0, 160, 1.5), torch.float32)]:
    x = torch.from_numpy(inputs.phantom_batch(7, 19, 96)).cuda().to(dt)
    y = op.forward_raw(x)
    g = torch.from_numpy(inputs.randn((19,) + op.sinogram_shape, 8)).cuda().to(dt)
    b = op.backprojection_raw(g)
    torch.cuda.synchronize()
    np.save(sys.argv[2] + f"_{name}_y.npy", y.float().cpu().numpy())
    np.save(sys.argv[2] + f"_{name}_b.npy", b.float().cpu().numpy())
"""


def _run(tmp_path, tag, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    prefix = str(tmp_path / tag)
    print(f"[gpu-step] variant {tag} {env_extra}", flush=True)
    r = subprocess.run([sys.executable, "-c", _SCRIPT, ROOT, prefix], env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return {k: (np.load(f"{prefix}_{k}_y.npy"), np.load(f"{prefix}_{k}_b.npy")) for k in ("par", "par16", "fan")}


def test_all_variants_agree(tmp_path):
    base = _run(tmp_path, "default", {})
    for fi, fs, bi, ba, bs in [(8, 0, 16, 4, 0), (4, 1, 32, 4, 1), (4, 0, 16, 8, 1), (16, 1, 32, 8, 0),
                               (8, 1, 16, 8, 1), (4, 1, 64, 4, 1), (8, 0, 64, 8, 0)]:
        got = _run(tmp_path, f"v{fi}{fs}{bi}{ba}{bs}", {"RADON_FORCE_SHAPE": f"{fi},{fs},{bi},{ba},{bs}"})
        for k in base:
            yb, bb = base[k]
            yg, bg = got[k]
            # the forward's per-image arithmetic does not depend on the shape
            assert np.array_equal(yb, yg), (k, fi, fs, "forward")
            e = rel_l2(bg, bb)
            report(f"variant_{k}_{fi}{fs}{bi}{ba}", bp_rel_diff=e)
            assert e <= (1e-6 if k != "par16" else 2e-3), (k, bi, ba, e)


def test_autotune_prepare_and_parity(tmp_path):
    """radon_prepare autotunes (and writes the cache file); results stay at parity."""
    cache = tmp_path / "tune.txt"
    script = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2009_14788_amd import inputs
from paper_2009_14788_amd.radon import Radon
op = Radon(128, inputs.uniform_angles(90), 182)
op.prepare(torch.float32, 12)
print(op.plan_info(torch.float32, 12))
x = torch.from_numpy(inputs.phantom_batch(9, 12, 128)).cuda()
np.save(sys.argv[2], op.forward_raw(x).cpu().numpy())
"""
    env = dict(os.environ, RADON_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", script, ROOT, str(tmp_path / "y.npy")], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    print(r.stdout)
    lines = cache.read_text().strip().splitlines()
    # key, fwd variant/images/staging, bp variant/images/angles/staging, fwd tiling
    assert len(lines) == 1 and len(lines[0].split()) == 9
    assert lines[0].split()[0].endswith("_t0_b16")             # FP32, batch class 16
    assert 0 <= int(lines[0].split()[8]) < 4
    y = np.load(tmp_path / "y.npy")
    og = oracle.Geometry(128, inputs.uniform_angles(90), 182, 1.0)
    ref = oracle.forward(og, inputs.phantom_batch(9, 12, 128)[:2].astype(np.float64))
    e = rel_l2(y[:2], ref)
    report("autotuned_forward", rel_l2=e)
    assert e <= TOL_F32
    # a second process reads the cache instead of timing
    r2 = subprocess.run([sys.executable, "-c", script, ROOT, str(tmp_path / "y2.npy")], env=env,
                        capture_output=True, text=True, timeout=240)
    assert r2.returncode == 0, r2.stderr[-2000:]
    assert len(cache.read_text().strip().splitlines()) == 1
    assert np.array_equal(np.load(tmp_path / "y2.npy"), y)


@pytest.mark.parametrize("tiling,rows,angles", [(1, 7, 8), (2, 15, 8), (3, 11, 4)])
def test_tune_cache_selects_forward_tiling(tmp_path, tiling, rows, angles):
    """A tune-cache line naming a forward tiling (slab rows, angles per item) is what
    the next process uses: plan_info reports it, and the result stays at parity with
    the oracle."""
    script = r"""
import sys, json, numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2009_14788_amd import inputs
from paper_2009_14788_amd.radon import Radon
op = Radon(128, inputs.uniform_angles(90), 182)
op.prepare(torch.float32, 12)
print(json.dumps(op.plan_info(torch.float32, 12)))
x = torch.from_numpy(inputs.phantom_batch(9, 12, 128)).cuda()
np.save(sys.argv[2], op.forward_raw(x).cpu().numpy())
"""
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, RADON_TUNE_CACHE=str(cache))
    # learn the key from a first tuning run, then rewrite its line with the tiling
    r = subprocess.run([sys.executable, "-c", script, ROOT, str(tmp_path / "y0.npy")], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    f = cache.read_text().split()
    f[1:4] = ["1", "8", "1"]                                    # tiled forward, 8 images, staged
    f[8] = str(tiling)
    cache.write_text(" ".join(f) + "\n")
    print(f"[gpu-step] tune cache forcing tiling {tiling}", flush=True)
    r = subprocess.run([sys.executable, "-c", script, ROOT, str(tmp_path / "y.npy")], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    info = json.loads(r.stdout.strip().splitlines()[-1])["forward"]
    assert (info["rows"], info["angles"], info["images"]) == (rows, angles, 8), info
    y = np.load(tmp_path / "y.npy")
    og = oracle.Geometry(128, inputs.uniform_angles(90), 182, 1.0)
    ref = oracle.forward(og, inputs.phantom_batch(9, 12, 128)[[0, 11]].astype(np.float64))
    e = rel_l2(y[[0, 11]], ref)
    report(f"tiling{tiling}_forward", rel_l2=e, rows=rows, angles=angles)
    assert e <= TOL_F32


def test_measure_peaks_plausible():
    """The device calibration returns finite rates within a broad plausible band for one
    MI355X-class GPU (multiply-adds per second and LDS bytes per second)."""
    import ctypes
    from paper_2009_14788_amd import _lib
    f, l = ctypes.c_double(0.0), ctypes.c_double(0.0)
    assert _lib.lib.radon_measure_peaks(ctypes.byref(f), ctypes.byref(l)) == 0
    print(f"[parity] device_peaks fma_per_s={f.value:.3e} lds_bytes_per_s={l.value:.3e}", flush=True)
    assert 1e12 < f.value < 1e15
    assert 1e12 < l.value < 1e15
