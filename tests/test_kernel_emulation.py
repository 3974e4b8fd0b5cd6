"""CPU checks of the kernels themselves: the library's HIP sources (kernels, planners,
ABI) are compiled for the host against a small emulation of the HIP runtime
(tests/emu/hip) with AddressSanitizer, so every kernel runs on the CPU with exact-size
buffers and LDS.  Any out-of-bounds access of a kernel fails these tests, and the
results are compared with the FP64 oracle (same bars as on the GPU) and with the
direct kernels; uneven batches are compared with the per-call results bitwise."""
import concurrent.futures
import math
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_2009_14788_amd import inputs
from _helpers import TOL_F32, TOL_16

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_14788_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
CLANG = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
         "-ffp-contract=off", "-pthread", "-w"]

pytestmark = pytest.mark.skipif(not os.path.exists(CLANG), reason="host clang++ not available")


@pytest.fixture(scope="module")
def emu_bin(tmp_path_factory):
    d = tmp_path_factory.mktemp("emu")
    src = d / "src"
    src.mkdir()
    for name in os.listdir(CSRC):
        text = open(os.path.join(CSRC, name)).read()
        if name == "radon_lds_dma.hpp":     # the asm-issued copy, emulated on the host
            text = open(os.path.join(EMU, "radon_lds_dma.hpp")).read()
        text = text.replace('"../../include/radon.h"', '"radon.h"')
        # dynamic LDS becomes the emulated block's buffer
        text = re.sub(r"extern __shared__ (\w+) (\w+)\[\];", r"\1 *\2 = (\1 *)emu::dyn_lds();", text)
        (src / name).write_text(text)
    inc = ["-I" + EMU, "-I" + os.path.join(ROOT, "include"), "-I" + str(src)]
    jobs = [[CLANG, *FLAGS, *inc, "-x", "c++", "-c", str(src / n), "-o", str(d / (n + ".o"))]
            for n in sorted(os.listdir(src)) if n.endswith((".cpp", ".hip"))]
    jobs.append([CLANG, "-x", "c", "-O1", "-g", "-fsanitize=address", "-ffp-contract=off", "-w", "-c",
                 os.path.join(ROOT, "oracle", "radon_oracle.c"), "-o", str(d / "oracle.o")])
    jobs.append([CLANG, *FLAGS, *inc, "-c", os.path.join(EMU, "emu_check.cpp"), "-o",
                 str(d / "emu_check.o")])
    with concurrent.futures.ThreadPoolExecutor(8) as ex:
        for r in ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), jobs):
            assert r.returncode == 0, r.stderr[-3000:]
    exe = d / "emu_check"
    objs = sorted(str(p) for p in d.glob("*.o"))
    r = subprocess.run([CLANG, *FLAGS, *objs, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _line(beam, n, angles, D, sp=1.0, S=0.0, E=0.0, step=1.0, batch=1, dt=0):
    ang = [float(a) for a in np.asarray(angles, dtype=np.float64).ravel()]
    return (f"{1 if beam == 'fan' else 0} {n} {D} {sp!r} {S!r} {E!r} {step!r} {batch} {dt} "
            f"{len(ang)} " + " ".join(repr(a) for a in ang))


def _run(exe, tmp_path, lines, mode="single", env=None):
    geo = tmp_path / "geos.txt"
    geo.write_text("\n".join(lines) + "\n")
    e = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    e.pop("RADON_VARIANT", None)
    e.update(env or {})
    r = subprocess.run([str(exe), str(geo), mode], capture_output=True, text=True, env=e,
                       timeout=900)
    assert "AddressSanitizer" not in r.stderr or "ERROR" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    rows = []
    for m in re.finditer(r"geometry (\d+) fwd_variant (\d) bp_variant (\d) forward (\S+) "
                         r"backprojection (\S+) direct_forward (\S+) direct_backprojection (\S+)",
                         r.stdout):
        rows.append((int(m.group(2)), int(m.group(3))) + tuple(float(m.group(i)) for i in range(4, 8)))
    assert len(rows) == len(lines), r.stdout
    return rows, r.stdout


def _check_bars(rows, lines):
    for (fv, bv, ef, eb, df, db), line in zip(rows, lines):
        tol = TOL_F32 if line.split()[8] == "0" else TOL_16
        assert max(ef, eb, df, db) <= tol, (line[:60], ef, eb, df, db)


def test_emulated_kernels_match_oracle(emu_bin, tmp_path):
    """Ragged, degenerate and 16-bit geometries of both beams: no out-of-bounds access,
    tiled and direct kernels within the parity bars of the oracle."""
    U = inputs.uniform_angles
    ang = [-0.3, 0.0, math.pi / 2, 1.234, 3 * math.pi, 7.5, -2.0]
    lines = [
        _line("par", 37, ang, 53, 0.8, step=0.7, batch=5),
        _line("fan", 37, ang, 53, 1.3, 70.0, 31.0, step=0.7, batch=5),
        _line("par", 64, U(64), 91),
        _line("fan", 64, U(64, 2 * math.pi), 91, 1.5, 120.0, 60.0),
        _line("fan", 48, U(40, 2 * math.pi), 70, 1.5, 400.0, 200.0, batch=2),
        _line("par", 1, [0.3], 1, batch=3),
        _line("fan", 1, [0.0, 1.0, 2.0], 5, 1.0, 10.0, 4.0, batch=3),
        _line("par", 2, [0.7], 1, batch=3),
        _line("par", 5, [0.0], 40, batch=3),
        _line("fan", 5, [0.0], 40, 1.0, 10.0, 4.0, batch=3),
        _line("par", 48, U(36), 70, batch=3, dt=1),
        _line("par", 48, U(36), 70, batch=3, dt=2),
        _line("fan", 48, U(36, 2 * math.pi), 70, 1.5, 250.0, 125.0, batch=3, dt=2),
    ]
    rows, _ = _run(emu_bin, tmp_path, lines)
    _check_bars(rows, lines)
    # the tiled kernels really ran on the regular geometries
    assert rows[2][:2] == (1, 1) and rows[10][:2] == (1, 1), rows


@pytest.mark.parametrize("shape", ["8,0,16,4,0", "4,1,32,4,1", "16,1,32,8,0", "8,1,16,8,1", "4,1,64,4,1",
                                   "8,0,64,8,0", "8,1,4,8,1", "4,0,4,4,0", "8,2,16,4,2", "16,2,32,8,0",
                                   "8,1,64,8,2", "16,2,8,4,2", "8,1,32,4,1,1", "4,0,16,8,0,2",
                                   "16,2,64,4,2,3", "8,1,64,8,1,3", "16,1,32,4,1,2", "16,1,64,4,1,1",
                                   "16,0,16,8,0,0", "8,2,64,2,2", "16,1,32,2,1", "8,1,16,2,0"])
def test_emulated_launch_shapes(emu_bin, tmp_path, shape):
    """Every forced launch shape (images per lane, staging -- 2: 16-bit tap pairs with
    dot2, forward or backprojection --, angle block -- fan beam 4 or 2 --, forward
    tiling: slab rows and angles per item) stays in bounds and at parity, with a ragged
    batch of 11 images and an angle count that leaves a partial angle block."""
    U = inputs.uniform_angles
    lines = [_line("par", 40, U(24), 57, batch=11),
             _line("par", 40, U(24), 57, batch=11, dt=1),
             _line("fan", 40, U(24, 2 * math.pi), 66, 1.5, 250.0, 120.0, batch=11),
             _line("fan", 37, U(24, 2 * math.pi), 60, 1.5, 250.0, 120.0, batch=11, dt=2),
             # source close enough that some tiles need 5-6 candidate bins (second pass)
             _line("fan", 40, U(16, 2 * math.pi), 80, 1.0, 130.0, 40.0, batch=11, dt=1),
             _line("fan", 36, U(23, 2 * math.pi), 60, 1.5, 250.0, 120.0, batch=11, dt=2)]
    rows, _ = _run(emu_bin, tmp_path, lines, env={"RADON_FORCE_SHAPE": shape})
    _check_bars(rows, lines)


@pytest.mark.parametrize("shape", ["8,2,16,4,2", "16,2,64,4,2"])
def test_emulated_tap_pairs_wide_windows(emu_bin, tmp_path, shape):
    """16-bit tap pairs where the forward's slab windows are wider than the fixed LDS
    pitch (bins 2 pixels apart at the isocentre, so 64 bins span ~130 columns and the
    run-time pitch is used), FP16 and BF16, ragged batch of 5."""
    U = inputs.uniform_angles
    lines = [_line("fan", 160, U(6, 2 * math.pi), 100, 3.0, 400.0, 200.0, batch=5, dt=1),
             _line("fan", 160, U(6, 2 * math.pi), 100, 3.0, 400.0, 200.0, batch=5, dt=2)]
    rows, _ = _run(emu_bin, tmp_path, lines, env={"RADON_FORCE_SHAPE": shape})
    _check_bars(rows, lines)
    assert all(r[0] == 1 for r in rows), rows


def test_emulated_uneven_batch_groups(emu_bin, tmp_path):
    """Jobs of different sizes, two sharing one geometry (their images share lanes),
    batch sizes 1..3: the batched launches equal the per-call results bitwise."""
    U = inputs.uniform_angles
    lines = [_line("par", 40, U(20), 57, batch=1),
             _line("par", 24, U(30, 2 * math.pi / 3), 34, batch=2),
             _line("par", 40, U(20), 57, batch=3),
             _line("fan", 32, U(16, 2 * math.pi), 46, 1.5, 200.0, 100.0, batch=1),
             _line("par", 56, U(12), 80, batch=1)]
    rows, out = _run(emu_bin, tmp_path, lines, mode="batched")
    _check_bars(rows, lines)
    assert "identical 5 of 5" in out, out


@pytest.mark.parametrize("dt", [1, 2])
def test_emulated_uneven_batch_16bit(emu_bin, tmp_path, dt):
    """16-bit uneven batch: the forward runs on tap pairs along x staged from the callers'
    images (four images per lane, including a ragged group of one and a fan job), within
    the 16-bit bar of the oracle; the backprojection is bitwise equal to per-call."""
    # the emulator prints each 16-bit batched forward's error against the oracle and
    # counts a job as matching only within 5e-3
    U = inputs.uniform_angles
    lines = [_line("par", 40, U(20), 57, batch=1, dt=dt),
             _line("par", 24, U(30, 2 * math.pi / 3), 34, batch=2, dt=dt),
             _line("par", 40, U(20), 57, batch=4, dt=dt),
             _line("fan", 32, U(16, 2 * math.pi), 46, 1.5, 200.0, 100.0, batch=1, dt=dt),
             _line("par", 37, U(9), 53, batch=3, dt=dt)]
    rows, out = _run(emu_bin, tmp_path, lines, mode="batched")
    print("\n".join(l for l in out.splitlines() if l.startswith("batched")))
    _check_bars(rows, lines)
    assert "identical 5 of 5" in out, out


def test_emulated_filter_matches_oracle(emu_bin, tmp_path):
    """The FBP filter kernel (Stockham radix-8/radix-4 transforms in LDS, two rows per
    block) against the FP64 oracle filter for all five filters: odd row counts, padded
    lengths 64 .. 8192 (every pass sequence), 16-bit storage."""
    from oracle import filtering
    U = inputs.uniform_angles
    specs = [("par", 16, U(7), 23, 1.0, 3, 0), ("par", 24, U(6), 91, 0.5, 1, 0),
             ("par", 20, U(5), 33, 1.0, 2, 1), ("par", 20, U(5), 40, 1.5, 1, 2),
             ("par", 8, U(3), 300, 1.0, 1, 0), ("par", 8, U(1), 1500, 1.0, 1, 0),
             ("par", 8, U(1), 2100, 1.0, 1, 0)]
    lines = [_line(b, n, a, D, sp, batch=B, dt=dt) for b, n, a, D, sp, B, dt in specs]
    geo = tmp_path / "geos.txt"
    geo.write_text("\n".join(lines) + "\n")
    dump = tmp_path / "filter.bin"
    r = subprocess.run([str(emu_bin), str(geo), "filter", str(dump)], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"), timeout=900)
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    data = np.fromfile(dump, dtype=np.float64)
    pos = 0
    for _, n, a, D, sp, B, dt in specs:
        A = len(a)
        size = B * A * D
        y = data[pos:pos + size].reshape(B, A, D)
        pos += size
        for name in filtering.FILTERS:
            got = data[pos:pos + size].reshape(B, A, D)
            pos += size
            ref = filtering.filter_sinogram(y, name)
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert err <= (TOL_F32 if dt == 0 else TOL_16), (n, D, dt, name, err)
    assert pos == data.size


def test_emulated_solvers_match_oracle(emu_bin, tmp_path):
    """The solver loops (radon_landweber, radon_cgne) and the per-system inner products,
    run through the emulated kernels: a few iterations of each, every batch entry its
    own system, against the FP64 oracle solvers on the same inputs."""
    import oracle
    from oracle import solvers
    U = inputs.uniform_angles
    specs = [("par", 24, U(20), 35, 1.0, 0.0, 0.0, 3), ("fan", 20, U(16, 2 * math.pi), 30, 1.5, 100.0, 50.0, 2)]
    lines = [_line(b, n, a, D, sp, S, E, batch=B) for b, n, a, D, sp, S, E, B in specs]
    geos = [oracle.Geometry(n, a, D, sp, beam=oracle.FANBEAM if b == "fan" else oracle.PARALLEL,
                            source_distance=S, det_distance=E) for b, n, a, D, sp, S, E, B in specs]
    iters = 3
    # a step below 2 / ||R||^2 (both systems share it; the value only has to agree)
    alpha = 1.0 / max(np.linalg.norm(oracle.dense_matrix(g), 2) ** 2 for g in geos)
    geo = tmp_path / "geos.txt"
    geo.write_text("\n".join(lines) + "\n")
    dump = tmp_path / "solver.bin"
    r = subprocess.run([str(emu_bin), str(geo), "solver", str(dump), repr(float(alpha)), str(iters)],
                       capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"), timeout=900)
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    data = np.fromfile(dump, dtype=np.float64)
    pos = 0

    def take(shape):
        nonlocal pos
        size = int(np.prod(shape))
        out = data[pos:pos + size].reshape(shape)
        pos += size
        return out

    for (b, n, a, D, sp, S, E, B), g in zip(specs, geos):
        x0, y = take((B, n, n)), take((B, len(a), D))
        lw, cg_ne, dots = take((B, n, n)), take((B, n, n)), take((B,))
        fwd = lambda v: oracle.forward(g, v)
        bp = lambda v: oracle.backproject(g, v)
        ref_lw = solvers.landweber(fwd, bp, y, alpha, iters, x0)[-1]
        e_lw = np.linalg.norm(lw - ref_lw) / np.linalg.norm(ref_lw)
        for k in range(B):
            ref_cg = solvers.cgne(fwd, bp, y[k], x0[k], iters)[-1]
            e_cg = np.linalg.norm(cg_ne[k] - ref_cg) / np.linalg.norm(ref_cg)
            assert e_cg <= TOL_F32, (b, k, e_cg)
        assert e_lw <= TOL_F32, (b, e_lw)
        ref_dots = np.einsum("kij,kij->k", x0, x0)
        assert np.allclose(dots, ref_dots, rtol=1e-12, atol=0), (dots, ref_dots)
    assert pos == data.size


def test_emulated_graph_lifetime_and_streams(emu_bin, tmp_path):
    """Uneven-batch tables and FP64 inner-product scratch under stream capture: a job
    list captured on two streams gives each stream its own work counter (and each
    inner product its own partials), a captured table survives 40 later job lists
    that push it out of the cache (its replay equals the eager result bitwise, with no
    use after free), two replays run at the same time, and nothing is allocated while
    a stream captures."""
    U = inputs.uniform_angles
    lines = [_line("par", 40, U(24), 57, batch=3), _line("par", 33, U(17, 2.0), 48, batch=2),
             _line("fan", 32, U(20, 2 * math.pi), 46, 1.5, 90.0, 45.0, batch=2)]
    geo = tmp_path / "geos.txt"
    geo.write_text("\n".join(lines) + "\n")
    r = subprocess.run([str(emu_bin), str(geo), "lifetime"], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"), timeout=900)
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    checks = dict(re.findall(r"check (\S+) (\S+)", r.stdout))
    assert set(checks) >= {"eager_status", "capture_status", "streams_use_own_counters",
                           "replay_after_eviction", "concurrent_replays",
                           "dot_streams_use_own_partials", "dot_concurrent_replays",
                           "no_allocation_under_capture", "noalloc_dot_equals_dot",
                           "noalloc_dot_rejects_oversize"}, r.stdout
    assert all(v == "ok" for v in checks.values()), r.stdout


@pytest.mark.parametrize("dt", [0, 2])
def test_emulated_shearlet_matches_oracle(emu_bin, tmp_path, dt):
    """The alpha-shearlet forward and adjoint kernels (filters built by the library's
    host code) through the emulation: square and non-square images, a ragged batch of 3
    over the column tiles, against the FP64 oracle on the same (storage-rounded) inputs;
    every access in bounds."""
    from oracle import shearlets as osh
    specs = [(64, 64, 3, [0.5, 0.5, 0.5]), (32, 128, 2, [0.5, 0.25]), (16, 16, 1, [0.5])]
    spec = tmp_path / "sh.txt"
    spec.write_text("".join(f"{w} {h} {b} {dt} {len(a)} " + " ".join(repr(x) for x in a) + "\n"
                            for w, h, b, a in specs))
    dump = tmp_path / "sh.bin"
    r = subprocess.run([str(emu_bin), str(spec), "shearlet", str(dump)], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"), timeout=900)
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    data = np.fromfile(dump, dtype=np.float64)
    pos = 0
    tol = TOL_F32 if dt == 0 else TOL_16
    for w, h, b, a in specs:
        psi = osh.filters(w, h, a)
        M = psi.shape[0]
        x = data[pos:pos + b * h * w].reshape(b, h, w); pos += b * h * w
        c = data[pos:pos + b * M * h * w].reshape(b, M, h, w); pos += b * M * h * w
        d = data[pos:pos + b * M * h * w].reshape(b, M, h, w); pos += b * M * h * w
        y = data[pos:pos + b * h * w].reshape(b, h, w); pos += b * h * w
        ec = np.linalg.norm(c - osh.forward(x, psi)) / np.linalg.norm(osh.forward(x, psi))
        ref = osh.adjoint(d, psi)
        ey = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        assert ec <= tol and ey <= tol, (w, h, ec, ey)
    assert pos == data.size
