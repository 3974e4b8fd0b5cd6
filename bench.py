#!/usr/bin/env python3
"""Throughput benchmark: forward projection + backprojection of 128 x 512^2 FP32
phantoms, 720 angles over [0, pi), 724 detector bins of spacing 1 (parallel beam).

One step = radon_forward of the whole batch followed by radon_backproject of the
resulting sinograms, inputs resident in GPU memory.  Prints ONE JSON line:
projections/s (images x angles per second through forward+backprojection), rays/s,
algorithmic HBM GB/s, the roofline of the dominant kernel (timed with HIP events on
the stream the kernels run on), and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick] [--no-solvers]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+backproj projections/s & rays/s, 512², 720 angles, batch 128; HBM GB/s"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_batch128_512.md")
COUNTER_RECORD = os.path.join(ROOT, "profiles", "cache_hit_rates_batch128_512_f32.md")


# the sources that define the forward and backprojection kernels, their launches and
# their work plans: the HBM traffic record is valid while these are unchanged
PROJECTOR_SOURCES = ("radon_abi.cpp", "radon_bp.hip", "radon_common.hpp", "radon_fwd.hip",
                     "radon_fwd_tiled.hpp", "radon_fwd_t0.hip", "radon_fwd_t1.hip", "radon_fwd_t2.hip",
                     "radon_fwd_t3.hip", "radon_launch.hpp", "radon_lds_dma.hpp", "radon_plan.hpp",
                     "radon_planner.cpp",
                     "radon_tiles.hpp")


def kernel_sources_sha256():
    """SHA-256 over the projector kernel and planner sources (name + bytes, sorted)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2009_14788_amd", "csrc")
    for name in sorted(PROJECTOR_SOURCES):
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _record_fields(path, tag):
    """The "<direction>:<launch shape>=<value>" fields of a committed counter record,
    or None when there is no record or the kernel sources changed since the counters
    were taken."""
    import re
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(tag + r" sources_sha256=(\w+) (.*?)-->", text)
    if not m or m.group(1) != kernel_sources_sha256():
        return None
    return dict(kv.split("=", 1) for kv in m.group(2).split())


def shape_key(info):
    """Launch shape of one direction as the counter records key it: variant, images
    per lane, angles per item or block, staging, and the forward's slab rows."""
    key = f"{info['variant']},{info['images']},{info['angles']},{info['staging']}"
    return key + (f",{info['rows']}" if "rows" in info else "")


def recorded_traffic(direction, shape):
    """HBM bytes per launch of one direction and launch shape from the committed
    counter record, or None when there is no record, the shape was not recorded, or
    the kernel sources changed since the counters were taken."""
    fields = _record_fields(TRAFFIC_RECORD, "traffic-record")
    v = (fields or {}).get(f"{direction}:{shape}")
    return int(v) if v is not None else None


def recorded_cache_counters(direction, shape):
    """L2 and vector-L1 hit rates and the LDS bank-conflict fraction of one direction's
    main kernel at one launch shape, from the committed counter record; None under the
    same conditions as the traffic record."""
    fields = _record_fields(COUNTER_RECORD, "counter-record")
    v = (fields or {}).get(f"{direction}:{shape}")
    if v is None:
        return None
    return {k: float(x) for k, x in (kv.split(":") for kv in v.split(","))}


def support_samples(n, angles, det_count, spacing, step, beam="parallel", S=0.0, E=0.0):
    """Number of (ray, k) samples inside the open support box |P| < (N+1)/2 of the
    bilinear interpolant, i.e. the samples a ray-driven projector must evaluate
    (per image, per direction).  Closed-form ray/box clipping in FP64."""
    th = np.asarray(angles, dtype=np.float64)[:, None]
    s = (np.arange(det_count) - 0.5 * (det_count - 1))[None, :] * spacing
    ux, uy = np.cos(th), np.sin(th)
    vx, vy = -uy, ux
    if beam == "parallel":
        fx, fy, wx, wy = s * ux, s * uy, vx + 0 * s, vy + 0 * s
    else:
        srcx, srcy = -S * vx, -S * vy
        ex, ey = E * vx + s * ux, E * vy + s * uy
        wx, wy = ex - srcx, ey - srcy
        L = np.hypot(wx, wy)
        wx, wy = wx / L, wy / L
        al = srcx * wx + srcy * wy
        fx, fy = srcx - al * wx, srcy - al * wy
    b = 0.5 * (n + 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        tlo = np.full(fx.shape, -np.inf)
        thi = np.full(fx.shape, np.inf)
        for f, w in ((fx, wx), (fy, wy)):
            t1 = np.where(w != 0, (-b - f) / w, np.where(np.abs(f) < b, -np.inf, np.inf))
            t2 = np.where(w != 0, (b - f) / w, np.where(np.abs(f) < b, np.inf, -np.inf))
            tlo = np.maximum(tlo, np.minimum(t1, t2))
            thi = np.minimum(thi, np.maximum(t1, t2))
    cnt = np.floor(thi / step - 1e-12) - np.ceil(tlo / step + 1e-12) + 1
    cnt = np.where(thi > tlo, np.maximum(cnt, 0), 0)
    return float(cnt.sum())


def cpu_model():
    """The host CPU's model name (first "model name" line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_proj_rate(og, x, batch_angles):
    """Projections/s of the FP64 oracle's forward + backprojection of the images x."""
    import oracle
    t0 = time.perf_counter()
    y = oracle.forward(og, x)
    t1 = time.perf_counter()
    oracle.backproject(og, y)
    t2 = time.perf_counter()
    return batch_angles / (t2 - t0), t1 - t0, t2 - t1


def cpu_baseline(angles, n, det_count, x_np):
    """The FP64 oracle (forward ray loop + scatter backprojection, OpenMP) on the host:
    the headline on a bounded sample, on every thread the oracle has and on one thread,
    plus the single 64^2 image, the 16 x 256^2 batch and the 200 uneven jobs in full."""
    import oracle
    from paper_2009_14788_amd import inputs
    threads = oracle.num_threads()
    og = oracle.Geometry(n, angles, det_count, 1.0)
    k = 8                                                      # images of the headline sample
    rate_all, tf, tb = _oracle_proj_rate(og, x_np[:k].astype(np.float64), k * len(angles))
    # one thread: one image at every 8th angle (the per-projection work does not depend
    # on the angle's position in the list)
    sub = np.asarray(angles)[::8]
    og1 = oracle.Geometry(n, sub, det_count, 1.0)
    oracle.set_num_threads(1)
    try:
        rate_one, _, _ = _oracle_proj_rate(og1, x_np[:1].astype(np.float64), len(sub))
        w0 = inputs.WORKLOADS["single64"]
        og0 = oracle.Geometry(64, w0.angles(), 91, 1.0)
        x0 = inputs.phantom(64, 10, [0, 0])[0][None].astype(np.float64)
        rate0_one, _, _ = _oracle_proj_rate(og0, x0, 64)
    finally:
        oracle.set_num_threads(threads)
    rate0_all, _, _ = _oracle_proj_rate(og0, x0, 64)
    w1 = inputs.WORKLOADS["batch16_256"]
    og1 = oracle.Geometry(256, w1.angles(), 363, 1.0)
    rate1, _, _ = _oracle_proj_rate(og1, inputs.phantom_batch(1, 16, 256).astype(np.float64), 16 * 256)
    jobs = inputs.uneven_jobs(200)
    t0 = time.perf_counter()
    for j in jobs:
        ogj = oracle.Geometry(j.n, j.angles(), j.det_count, 1.0)
        oracle.backproject(ogj, oracle.forward(ogj, inputs.uneven_phantom(j)[None].astype(np.float64)))
    t3 = time.perf_counter() - t0
    return {
        "value": round(rate_all, 1), "unit": "projections/s", "cores": int(threads), "kind": "oracle",
        "sample": f"{k} of the 128 images at all {len(angles)} angles, forward + backprojection "
                  f"(FP64; forward {tf:.2f} s, backprojection {tb:.2f} s on {threads} threads)",
        "threads": int(threads), "cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
        "all_core_proj_s": round(rate_all, 1),
        "single_thread_proj_s": round(rate_one, 1),
        "single_thread_sample": f"1 image at {len(sub)} of the 720 angles (every 8th)",
        "workloads_full": {
            "single64": {"all_core_proj_s": round(rate0_all, 1), "single_thread_proj_s": round(rate0_one, 1)},
            "batch16_256": {"all_core_proj_s": round(rate1, 1)},
            "uneven200": {"all_core_proj_s": round(sum(j.n_angles for j in jobs) / t3, 1),
                          "seconds": round(t3, 2)},
        },
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true",
                    help="only the headline workload (skip the other workloads and forms)")
    ap.add_argument("--no-solvers", action="store_true",
                    help="leave out the Landweber / CGNE workloads (2 x 500 iterations of "
                         "several thousand dispatches, which dominate a counter-collection run)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the benchmark, run a plain elementwise copy of 1 GiB three times "
                         "(reference dispatch for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (the transform is single-GPU; batch sharding "
              "across GPUs is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_14788_amd import inputs
    from paper_2009_14788_amd.radon import Radon

    w = inputs.WORKLOADS["batch128_512"]
    B, N, A, D = w.batch, w.n, w.n_angles, w.det_count
    angles = w.angles()
    print(f"[bench] building {B} phantoms {N}x{N}", file=sys.stderr, flush=True)
    x_np = inputs.phantom_batch(2, B, N)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x = torch.from_numpy(x_np).to(dev)
    op = Radon(N, angles, D, 1.0)
    op.prepare(torch.float32, B)
    stream = torch.cuda.current_stream(dev)

    def step(xin):
        y = op.forward_raw(xin)
        xb = op.backprojection_raw(y)
        return y, xb

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step(x)
    torch.cuda.synchronize()

    # timed region: K steps; per-kernel HIP events on the launch stream
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        y = op.forward_raw(x)
        ev[i][1].record(stream)
        op.backprojection_raw(y)
        ev[i][2].record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = start.elapsed_time(end) / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    bp_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    print(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step (forward {fwd_ms:.3f} ms, "
          f"backprojection {bp_ms:.3f} ms), host wall {wall:.3f} s", file=sys.stderr, flush=True)

    proj_s = B * A / (ms_step * 1e-3)
    rays_s = B * A * D / (ms_step * 1e-3)
    bytes_dir = 4.0 * B * (N * N + A * D)          # unique input + output, one direction
    hbm_gbs = 2 * bytes_dir / (ms_step * 1e-3) / 1e9
    samples = support_samples(N, angles, D, 1.0, 1.0) * B
    flop = 8.0 * samples                            # 4 multiply-adds per image-sample
    dom = "forward" if fwd_ms >= bp_ms else "backprojection"
    dom_ms = max(fwd_ms, bp_ms)
    achieved = flop / (dom_ms * 1e-3) / 1e12
    info = op.plan_info(torch.float32, B)[dom]
    shape = shape_key(info)
    kernels = {("forward", 1, 1): "interleave_images + fwd_tiled_il", ("forward", 1, 0): "fwd_tiled",
               ("backprojection", 1, 1): "interleave_sinograms + bp_tiled_par_il",
               ("backprojection", 1, 0): "bp_tiled_par"}.get(
                   (dom, info["variant"], info["staging"]), f"{dom}_direct")
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": recorded_traffic(dom, shape),
            "kernel": f"{dom}: {kernels}", "kernel_ms": round(dom_ms, 4), "shape": shape,
            "work": f"8 flop per (image, ray sample); {samples:.4e} samples per launch",
            "algorithmic_bytes": int(bytes_dir)}

    # per direction: throughput and the fractions of the device's measured FP32
    # multiply-add rate and LDS read bandwidth that the algorithm's own work reaches
    # (forward: 4 multiply-adds and 4 taps of 4 bytes per image-sample; backprojection:
    # 3 candidate bins, 3 multiply-adds and 3 x 4 bytes per image, pixel and angle)
    from paper_2009_14788_amd import _lib
    import ctypes
    fma_peak, lds_peak = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = _lib.lib.radon_measure_peaks(ctypes.byref(fma_peak), ctypes.byref(lds_peak))
    _lib.check("radon_measure_peaks", rc)
    fma_peak, lds_peak = fma_peak.value, lds_peak.value
    triples = float(B) * N * N * A

    def direction(ms, fmas, lds_bytes):
        t = ms * 1e-3
        return {"ms": round(ms, 4), "projections_per_s": round(B * A / t, 1),
                "rays_per_s": round(B * A * D / t, 1),
                "hbm_gbs_algorithmic": round(bytes_dir / t / 1e9, 2),
                "hbm_frac": round(bytes_dir / t / 1e9 / PEAK_HBM_GBS, 5),
                "fma_frac_of_measured": round(fmas / t / fma_peak, 4),
                "lds_frac_of_measured": round(lds_bytes / t / lds_peak, 4)}

    directions = {"forward": direction(fwd_ms, 4.0 * samples, 16.0 * samples),
                  "backprojection": direction(bp_ms, 3.0 * triples, 12.0 * triples)}
    for d in directions:
        directions[d]["counters"] = recorded_cache_counters(d, shape_key(op.plan_info(torch.float32, B)[d]))
    peaks = {"fma_per_s": fma_peak, "lds_bytes_per_s": lds_peak,
             "method": "radon_measure_peaks: v_fmac_f32 chains (packed FP32 off) and conflict-free "
                       "ds_read_b128 streams on this GPU, best of 3 runs"}

    # correctness of this very output against the oracle: whole images 0 and 127 (the
    # first and last lane of the image groups) of the forward, and of the backprojection
    # (same launch shape) of seeded N(0,1) sinograms
    import oracle
    og = oracle.Geometry(N, angles, D, 1.0)
    sel = [0, B - 1]
    yg = y[sel].double().cpu().numpy()
    yr = oracle.forward(og, x_np[sel].astype(np.float64))
    err = float(np.linalg.norm(yg - yr) / np.linalg.norm(yr))
    err_max = float(np.abs(yg - yr).max() / np.abs(yr).max())
    ys_np = inputs.randn((B, A, D), 2024)
    xb = op.backprojection_raw(torch.from_numpy(ys_np).to(dev))
    xg = xb[sel].double().cpu().numpy()
    del xb
    xr = oracle.backproject(og, ys_np[sel].astype(np.float64))
    err_bp = float(np.linalg.norm(xg - xr) / np.linalg.norm(xr))
    err_bp_max = float(np.abs(xg - xr).max() / np.abs(xr).max())

    out = {
        "metric": METRIC, "value": round(proj_s, 1), "unit": "projections/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch128_512", "beam": "parallel", "batch": B, "image_size": N,
                   "angles": A, "arc": "[0,pi)", "det_count": D, "det_spacing": 1.0,
                   "step_length": 1.0, "step": "forward + backprojection"},
        "rays_per_s": round(rays_s, 1), "hbm_gbs_algorithmic": round(hbm_gbs, 2),
        "hbm_frac": round(hbm_gbs / PEAK_HBM_GBS, 5),
        "forward_ms": round(fwd_ms, 4), "backprojection_ms": round(bp_ms, 4),
        "fwd_rel_l2_vs_oracle": err, "fwd_max_abs_over_max_ref": err_max,
        "bp_rel_l2_vs_oracle": err_bp, "bp_max_abs_over_max_ref": err_bp_max,
        "error_sample": "whole images 0 and 127; backprojection of seeded N(0,1) sinograms",
        "roofline": roof,
        "directions": directions,
        "device_peaks": peaks,
    }
    if not args.quick:
        ref = {"sel": sel, "y": yr, "ys": ys_np, "xb": xr}
        out["workloads"] = variants(op, x, x_np, B, A, D, ref, solvers=not args.no_solvers)
    if args.copy_calibration:
        # a plain elementwise kernel that reads 1 GiB once and writes 1 GiB once
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(angles, N, D, x_np)
    print(json.dumps(out), flush=True)


def _timed(fn, reps=5, warm=1):
    """Average ms of fn() over reps runs on the current stream (HIP events)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def _graph_ms(fn, reps=20):
    """Average ms per replay of fn() captured into a graph."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return _timed(g.replay, reps=reps, warm=2)


def _sampled_err(og, x_np, y_dev, n=16, seed=0):
    """Relative L2 error of n sampled forward outputs against the FP64 oracle."""
    import oracle
    B, A, D = y_dev.shape
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, B, n), rng.integers(0, A, n), rng.integers(0, D, n)], 1)
    yg = y_dev[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    yr = oracle.forward_rays(og, x_np, idx)
    return float(np.linalg.norm(yg - yr) / np.linalg.norm(yr))


def _bp_err(og, bp_fn, sino_shape, dt, seed, n_pix=16):
    """Relative L2 error of n_pix sampled backprojection outputs of seeded N(0,1)
    sinograms (stored in dt) against the FP64 oracle on the same FP32 values."""
    import oracle
    import torch
    ys = inputs_mod().randn(sino_shape, seed)
    xb = bp_fn(torch.from_numpy(ys).cuda().to(dt))
    Bn, N = xb.shape[0], xb.shape[-1]
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, Bn, n_pix), rng.integers(0, N, n_pix), rng.integers(0, N, n_pix)], 1)
    got = xb[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    ref = oracle.backproject_pixels(og, ys.astype(np.float64), idx)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def inputs_mod():
    from paper_2009_14788_amd import inputs
    return inputs


def _frac(samples, ms):
    """Fraction of the FP32 vector peak reached by forward + backprojection: 8 flop per
    image-sample in each direction."""
    return round(16.0 * samples / (ms * 1e-3) / (PEAK_FP32_TFLOPS * 1e12), 4)


def variants(op, x, x_np, B, A, D, ref, solvers=True):
    """The other workloads and forms, each timed on this GPU with its error stated:
    16-bit storage and the differentiable step on the headline batch; the single 64^2
    image (latency, eager and graph-replayed); the 16 x 256^2 batch; 200 uneven jobs
    in one persistent launch (eager, graph, and one call per job); the 64 x 512^2
    fan beam with 16-bit storage and a 10-step unrolled gradient descent
    differentiated end to end; the FBP filter on the headline sinograms, FBP in the
    paper's 512^2 configuration, and Landweber and CGNE (500 iterations) there (unless
    solvers is False)."""
    import math
    import torch
    import oracle
    from paper_2009_14788_amd import inputs
    from paper_2009_14788_amd.batched import BatchedRadon
    from paper_2009_14788_amd.radon import Radon, RadonFanbeam, dot_f64
    from paper_2009_14788_amd.solvers import Landweber, cgne, power_iteration, unrolled_gd
    res = {}
    og = oracle.Geometry(op.resolution, op.angles, D, 1.0)

    samples128 = support_samples(op.resolution, op.angles, D, 1.0, 1.0) * B

    # -- 16-bit storage on the headline batch (errors on whole images 0 and 127 against
    #    the oracle on the original FP32 values, storage rounding included)
    y32 = op.forward_raw(x)
    sel = ref["sel"]
    ys16 = torch.from_numpy(ref["ys"]).cuda()
    for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        xh = x.to(dt)
        op.prepare(dt, B)
        ms = _timed(lambda: op.backprojection_raw(op.forward_raw(xh)))
        yh = op.forward_raw(xh)
        yg = yh[sel].double().cpu().numpy()
        xbh = op.backprojection_raw(ys16.to(dt))[sel].double().cpu().numpy()
        res[f"batch128_512_{name}"] = {
            "ms_per_step": round(ms, 4), "projections_per_s": round(B * A / (ms * 1e-3), 1),
            "roofline_frac_fp32_peak": _frac(samples128, ms),
            "fwd_rel_l2_vs_f32_path": float((yh.float() - y32).norm() / y32.norm()),
            "fwd_rel_l2_vs_oracle": float(np.linalg.norm(yg - ref["y"]) / np.linalg.norm(ref["y"])),
            "bp_rel_l2_vs_oracle": float(np.linalg.norm(xbh - ref["xb"]) / np.linalg.norm(ref["xb"])),
            "error_sample": "whole images 0 and 127"}
        print(f"[bench] {name}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
        del xh, yh
    del ys16

    # -- differentiable step: loss ||R x - y||^2 (FP64 reduction), backward via R^T
    rng_noise = np.random.default_rng([2, 10 ** 6])
    ymeas = y32 + torch.from_numpy(
        (rng_noise.standard_normal(tuple(y32.shape)) * 0.01 *
         y32.amax(dim=(1, 2)).cpu().numpy()[:, None, None]).astype(np.float32)).cuda()
    xg = torch.zeros_like(x).requires_grad_(True)

    def ad_step():
        xg.grad = None
        r = op.forward(xg) - ymeas
        (r * r).sum().backward()
        return dot_f64(r.detach(), r.detach())

    ms = _timed(ad_step)
    res["batch128_512_autograd_loss_step"] = {
        "ms_per_step": round(ms, 4), "projections_per_s": round(B * A / (ms * 1e-3), 1),
        "note": "forward + loss + backward (transpose kernel) + FP64 loss reduction"}
    print(f"[bench] autograd loss step: {ms:.3f} ms", file=sys.stderr, flush=True)
    del ymeas, xg, y32

    # -- FBP (Sec. 3.1.3): the filter on the headline sinograms, and the paper's FBP
    #    configuration (512^2, 512 angles over [0, pi), ceil(512 sqrt 2) bins, Ram-Lak)
    y128 = op.forward_raw(x)
    ms_f = _timed(lambda: op.filter_sinogram_raw(y128, "ram-lak"))
    rows = B * A
    L = 1 << max(6, (2 * D - 1).bit_length())
    res["fbp_filter_batch128_512"] = {
        "ms_per_call": round(ms_f, 4), "projections_per_s": round(rows / (ms_f * 1e-3), 1),
        "padded_length": L,
        "note": "ram-lak filter of 128 x 720 rows of 724 bins (two rows per complex transform)"}
    print(f"[bench] fbp filter 128x720x724: {ms_f:.3f} ms", file=sys.stderr, flush=True)
    del y128
    Dp = int(math.ceil(math.sqrt(2) * 512))
    opf = Radon(512, inputs.uniform_angles(512), Dp)
    xf_np = inputs.phantom(512, 10, [12, 0])[0][None]
    xf = torch.from_numpy(xf_np).cuda()
    yf = opf.forward_raw(xf)
    ms_fbp = _timed(lambda: opf.backprojection_raw(opf.filter_sinogram_raw(yf, "ram-lak")), reps=20)
    rec = opf.backprojection_raw(opf.filter_sinogram_raw(yf, "ram-lak"))[0].double().cpu().numpy()
    rr = np.hypot(*(np.mgrid[0:512, 0:512] - 255.5))
    inside = rr < 248
    res["fbp_paper_512"] = {
        "ms_per_fbp": round(ms_fbp, 4),
        "mse_vs_phantom_inside": float(np.mean((rec[inside] - xf_np[0][inside]) ** 2)),
        "note": "filter + backprojection of one 512^2 sinogram (512 angles, 725 bins); random "
                "ellipses stand in for the paper's Shepp-Logan phantom (its MSE 2.22e-4 is on that)"}
    print(f"[bench] fbp 512^2 paper configuration: {ms_fbp:.3f} ms", file=sys.stderr, flush=True)

    # -- solvers (Sec. 4.2) in the same configuration: Landweber with alpha = 0.95 / ||R||^2
    #    from power iteration and CGNE, 500 iterations each from a zero guess
    lw = Landweber(opf)
    alpha = lw.estimate_alpha(512, "cuda") * 0.95
    zero = torch.zeros_like(xf)
    sol = {}
    runs = (("landweber", lambda it: lw.run(zero, yf, alpha, iterations=it)),
            ("cgne", lambda it: cgne(opf, zero, yf, max_iter=it))) if solvers else ()
    for name, run in runs:
        ms = _timed(lambda: run(500), reps=2)
        rec = run(500)[0].double().cpu().numpy()
        sol[name] = {"ms_per_iteration": round(ms / 500, 5), "ms_500_iterations": round(ms, 3),
                     "mse_vs_phantom": float(np.mean((rec - xf_np[0]) ** 2)),
                     "mse_vs_phantom_inside": float(np.mean((rec[inside] - xf_np[0][inside]) ** 2))}
        print(f"[bench] {name} 512^2 paper configuration: {ms / 500:.4f} ms/iteration",
              file=sys.stderr, flush=True)
    if solvers:
        res["solvers_paper_512"] = dict(sol, alpha=alpha, note=(
            "500 iterations from zero on one 512^2 phantom (512 angles, 725 bins), each loop "
            "queued natively with device-side FP64 scalars; random ellipses stand in for "
            "Shepp-Logan (the paper's MSEs 1.39e-4 Landweber, 4.42e-5 CGNE are on that)"))

    # -- single 64x64 image (latency)
    w0 = inputs.WORKLOADS["single64"]
    op0 = Radon(64, w0.angles(), 91)
    x0_np = inputs.phantom(64, 10, [0, 0])[0][None]
    x0 = torch.from_numpy(x0_np).cuda()
    op0.prepare(torch.float32, 1)
    eager = _timed(lambda: op0.backprojection_raw(op0.forward_raw(x0)), reps=50, warm=5)
    graph = _graph_ms(lambda: op0.backprojection_raw(op0.forward_raw(x0)), reps=100)
    og0 = oracle.Geometry(64, w0.angles(), 91, 1.0)
    e0 = float(np.linalg.norm(op0.forward_raw(x0)[0].double().cpu().numpy() - oracle.forward(og0, x0_np[0].astype(np.float64)))
               / np.linalg.norm(oracle.forward(og0, x0_np[0].astype(np.float64))))
    e0b = _bp_err(og0, lambda t: op0.backprojection_raw(t), (1, 64, 91), torch.float32, 5, n_pix=64)
    res["single64"] = {"us_per_step_eager": round(eager * 1e3, 2), "us_per_step_graph": round(graph * 1e3, 2),
                       "fwd_rel_l2_vs_oracle": e0, "bp_rel_l2_vs_oracle_sampled": e0b}

    # -- 16 x 256^2
    w1 = inputs.WORKLOADS["batch16_256"]
    op1 = Radon(256, w1.angles(), 363)
    x1_np = inputs.phantom_batch(1, 16, 256)
    x1 = torch.from_numpy(x1_np).cuda()
    op1.prepare(torch.float32, 16)
    ms = _timed(lambda: op1.backprojection_raw(op1.forward_raw(x1)), reps=20)
    og1 = oracle.Geometry(256, w1.angles(), 363, 1.0)
    res["batch16_256"] = {"ms_per_step": round(ms, 4), "projections_per_s": round(16 * 256 / (ms * 1e-3), 1),
                          "roofline_frac_fp32_peak": _frac(support_samples(256, w1.angles(), 363, 1.0, 1.0) * 16, ms),
                          "fwd_rel_l2_vs_oracle_sampled": _sampled_err(og1, x1_np, op1.forward_raw(x1), seed=2),
                          "bp_rel_l2_vs_oracle_sampled": _bp_err(og1, lambda t: op1.backprojection_raw(t),
                                                                 (16, 256, 363), torch.float32, 6)}

    # -- 200 uneven jobs in one persistent launch
    jobs = inputs.uneven_jobs(200)
    ops = [Radon(j.n, j.angles(), j.det_count, 1.0) for j in jobs]
    proj = sum(j.n_angles for j in jobs)
    samples_uneven = sum(support_samples(j.n, j.angles(), j.det_count, 1.0, 1.0) for j in jobs)
    br = BatchedRadon(ops)
    for name, dt in (("f32", torch.float32), ("f16", torch.float16)):
        xs = [torch.from_numpy(inputs.uneven_phantom(j)[None]).cuda().to(dt) for j in jobs]
        ys = [torch.empty((1,) + o.sinogram_shape, device="cuda", dtype=dt) for o in ops]
        bs = [torch.empty((1,) + o.image_shape, device="cuda", dtype=dt) for o in ops]

        def step():
            br.forward(xs, out=ys)
            br.backprojection(ys, out=bs)

        ms_e = _timed(step, reps=10)
        ms_g = _graph_ms(step, reps=10)
        ms_seq = _timed(lambda: [o.backprojection_raw(o.forward_raw(xx)) for o, xx in zip(ops, xs)], reps=3)
        # errors of whole jobs: every 20th job, forward of its phantom and backprojection
        # of seeded N(0,1) sinograms, in the same persistent launches
        gs = [torch.from_numpy(inputs.randn((1,) + o.sinogram_shape, 900 + i)).cuda().to(dt)
              for i, o in enumerate(ops)]
        br.forward(xs, out=ys)
        br.backprojection(gs, out=bs)
        ef = eb = 0.0
        for k in range(0, len(jobs), 20):
            jk = jobs[k]
            ogk = oracle.Geometry(jk.n, jk.angles(), jk.det_count, 1.0)
            yr = oracle.forward(ogk, inputs.uneven_phantom(jk)[None].astype(np.float64))
            ef = max(ef, float(np.linalg.norm(ys[k].double().cpu().numpy() - yr) / np.linalg.norm(yr)))
            br_ = oracle.backproject(ogk, gs[k].float().double().cpu().numpy())
            eb = max(eb, float(np.linalg.norm(bs[k].double().cpu().numpy() - br_) / np.linalg.norm(br_)))
        res[f"uneven200_{name}"] = {
            "ms_per_step_eager": round(ms_e, 4), "ms_per_step_graph": round(ms_g, 4),
            "ms_per_step_one_call_per_job": round(ms_seq, 4),
            "projections_per_s_graph": round(proj / (ms_g * 1e-3), 1),
            "roofline_frac_fp32_peak_graph": _frac(samples_uneven, ms_g),
            "samples_per_direction": samples_uneven,
            "fwd_rel_l2_vs_oracle_worst_job": ef, "bp_rel_l2_vs_oracle_worst_job": eb,
            "error_sample": "every 20th job, whole images"}
        print(f"[bench] uneven200 {name}: eager {ms_e:.3f} graph {ms_g:.3f} per-job {ms_seq:.3f} ms",
              file=sys.stderr, flush=True)
        del xs, ys, bs

    # -- fan beam 64 x 512^2, 16-bit storage; unrolled GD differentiated end to end.  The
    #    GD error is stated on image 0 against the oracle GD: the oracle's projection of
    #    the phantom as data (rounded to the storage type), a fixed step 0.95 / 5.2e5 shared
    #    by both sides (5.2e5 rounds up the power-iteration estimate of ||R||^2), per
    #    iteration, and the gradient of ||x_10 - x_true||^2 with respect to the data.
    from oracle import solvers as osolvers
    w4 = inputs.WORKLOADS["fan64_512"]
    op4 = RadonFanbeam(512, w4.angles(), 1000.0, 500.0, 1024, 1.5)
    x4_np = inputs.phantom_batch(4, 64, 512)
    og4 = oracle.Geometry(512, w4.angles(), 1024, 1.5, beam=oracle.FANBEAM, source_distance=1000.0,
                          det_distance=500.0)
    samples_fan = support_samples(512, w4.angles(), 1024, 1.5, 1.0, "fan", 1000.0, 500.0) * 64
    lam = power_iteration(op4)
    alpha = 1.0 / lam
    alpha_check = 0.95 / 5.2e5
    print("[bench] fan GD oracle (image 0)", file=sys.stderr, flush=True)
    xt0 = x4_np[:1].astype(np.float64)
    y0_ref = oracle.forward(og4, xt0)
    it_ref, grad_ref = osolvers.unrolled_gd_grad(lambda v: oracle.forward(og4, v),
                                                 lambda r: oracle.backproject(og4, r), y0_ref,
                                                 alpha_check, 10, xt0)
    from paper_2009_14788_amd.solvers import gd_step
    for name, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        x4 = torch.from_numpy(x4_np).cuda().to(dt)
        op4.prepare(dt, 64)
        ms = _timed(lambda: op4.backprojection_raw(op4.forward_raw(x4), scale=alpha), reps=5)
        y4 = op4.forward_raw(x4)
        e4 = _sampled_err(og4, x4_np, y4, seed=7)
        e4b = _bp_err(og4, lambda t: op4.backprojection_raw(t), (64, 1024, 1024), dt, 8)
        yreq = y4.clone().requires_grad_(True)

        def gd_backward():
            yreq.grad = None
            xk = unrolled_gd(op4, yreq, alpha, iters=10, checkpoint=True)
            ((xk.float() - x4.float()) ** 2).sum().backward()

        ms_gd = _timed(gd_backward, reps=2)
        # GD errors on image 0 (same batch of 64, data of image 0 from the oracle)
        ye = y4.clone()
        ye[0] = torch.from_numpy(y0_ref[0].astype(np.float32)).cuda().to(dt)
        errs = []
        with torch.no_grad():
            xk = torch.zeros_like(x4)
            for k in range(10):
                xk = gd_step(op4, xk, ye, alpha_check)
                errs.append(float(np.linalg.norm(xk[0].double().cpu().numpy() - it_ref[k][0])
                                  / np.linalg.norm(it_ref[k][0])))
        yr = ye.clone().requires_grad_(True)
        xk = unrolled_gd(op4, yr, alpha_check, iters=10, checkpoint=True)
        ((xk.float() - x4.float()) ** 2).sum().backward()
        g0 = yr.grad[0].double().cpu().numpy()
        e_grad = float(np.linalg.norm(g0 - grad_ref[0]) / np.linalg.norm(grad_ref[0]))
        res[f"fan64_512_{name}"] = {
            "ms_per_step": round(ms, 4), "projections_per_s": round(64 * 1024 / (ms * 1e-3), 1),
            "roofline_frac_fp32_peak": _frac(samples_fan, ms),
            "fwd_rel_l2_vs_oracle_sampled": e4, "bp_rel_l2_vs_oracle_sampled": e4b, "alpha": alpha,
            "unrolled_gd10_fwd_bwd_ms": round(ms_gd, 3),
            "gd10_iterate_rel_l2_vs_oracle": [round(e, 6) for e in errs],
            "gd10_grad_y_rel_l2_vs_oracle": e_grad,
            "gd_error_sample": f"image 0, step {alpha_check:.6e} on both sides"}
        print(f"[bench] fan {name}: {ms:.3f} ms/step, unrolled GD fwd+bwd {ms_gd:.1f} ms, "
              f"GD error x10 {errs[-1]:.2e} grad {e_grad:.2e}", file=sys.stderr, flush=True)
        del x4, y4, yreq, ye, yr

    # -- alpha-shearlet transform (Sec. 3.2 configuration: 512^2, alpha = 0.5, 5 scales,
    #    59 channels), a batch of 16 phantoms: forward, adjoint, and the error of image 0's
    #    coefficients against the FP64 oracle and of the reconstruction
    from oracle import shearlets as osh
    from paper_2009_14788_amd.shearlet import ShearletTransform
    sh = ShearletTransform(512, 512, [0.5] * 5)
    Bs = 16
    xs_np = inputs.phantom_batch(2, Bs, 512)
    xs = torch.from_numpy(xs_np).cuda()
    sh.prepare(Bs)
    ms_f = _timed(lambda: sh.forward_raw(xs), reps=5)
    cs = sh.forward_raw(xs)
    ms_a = _timed(lambda: sh.backward_raw(cs), reps=5)
    rec = sh.backward_raw(cs)
    psi = osh.filters(512, 512, [0.5] * 5)
    c0 = cs[0].double().cpu().numpy()
    c0r = osh.forward(xs_np[0].astype(np.float64), psi)
    rec_np = rec.double().cpu().numpy()
    bytes_dir = 4.0 * Bs * 512 * 512 * (1 + sh.channels)
    res["shearlet_512_a05_s5"] = {
        "batch": Bs, "channels": sh.channels,
        "forward_ms": round(ms_f, 4), "adjoint_ms": round(ms_a, 4),
        "images_per_s_forward": round(Bs / (ms_f * 1e-3), 1),
        "hbm_gbs_algorithmic_forward": round(bytes_dir / (ms_f * 1e-3) / 1e9, 1),
        "hbm_frac_forward": round(bytes_dir / (ms_f * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "hbm_frac_adjoint": round(bytes_dir / (ms_a * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "coeff_rel_l2_vs_oracle_image0": float(np.linalg.norm(c0 - c0r) / np.linalg.norm(c0r)),
        "reconstruction_rel_l2": float(np.linalg.norm(rec_np - xs_np) / np.linalg.norm(xs_np)),
        "note": "algorithmic bytes per direction: the images and the 59-channel coefficients, FP32"}
    print(f"[bench] shearlet 16 x 512^2: forward {ms_f:.3f} ms, adjoint {ms_a:.3f} ms",
          file=sys.stderr, flush=True)
    del cs, rec, xs
    return res


if __name__ == "__main__":
    main()
