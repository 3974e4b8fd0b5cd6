#!/usr/bin/env python3
"""Throughput benchmark: forward projection + backprojection of 128 x 512^2 FP32
phantoms, 720 angles over [0, pi), 724 detector bins of spacing 1 (parallel beam).

One step = radon_forward of the whole batch followed by radon_backproject of the
resulting sinograms, inputs resident in GPU memory.  Prints ONE JSON line:
projections/s (images x angles per second through forward+backprojection), rays/s,
algorithmic HBM GB/s, the roofline of the dominant kernel (timed with HIP events on
the stream the kernels run on), and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--variants]
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


def cpu_baseline(case_angles, n, det_count, x_np, max_threads=16):
    """FP64 oracle (forward + scatter backprojection) on the host cores, on a bounded
    sample: the first `threads` images of the batch at all angles."""
    import oracle
    threads = oracle.num_threads()
    k = max(1, min(threads, max_threads, x_np.shape[0]))
    og = oracle.Geometry(n, case_angles, det_count, 1.0)
    xs = x_np[:k].astype(np.float64)
    t0 = time.perf_counter()
    y = oracle.forward(og, xs)
    t1 = time.perf_counter()
    oracle.backproject(og, y)
    t2 = time.perf_counter()
    proj = k * len(case_angles)
    return {
        "value": proj / (t2 - t0), "unit": "projections/s", "cores": int(min(threads, k)),
        "kind": "oracle",
        "sample": f"{k} of the 128 images, all {len(case_angles)} angles, forward + backprojection "
                  f"(FP64, OpenMP over images x angles / images); forward {t1 - t0:.2f} s, "
                  f"backprojection {t2 - t1:.2f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--variants", action="store_true",
                    help="also time FP16/BF16 storage and the autograd step")
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
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": dom, "kernel_ms": round(dom_ms, 4),
            "work": f"8 flop per (image, ray sample); {samples:.4e} samples per launch"}

    # sampled correctness of this very output against the oracle (8 rays)
    import oracle
    og = oracle.Geometry(N, angles, D, 1.0)
    rng = np.random.default_rng(0)
    idx = np.stack([rng.integers(0, B, 8), rng.integers(0, A, 8), rng.integers(0, D, 8)], 1)
    yg = y[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    yr = oracle.forward_rays(og, x_np, idx)
    err = float(np.linalg.norm(yg - yr) / np.linalg.norm(yr))

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
        "sampled_rel_l2_vs_oracle": err,
        "roofline": roof,
    }
    if args.variants:
        out["variants"] = variants(op, x, B, A, D)
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(angles, N, D, x_np)
    print(json.dumps(out), flush=True)


def variants(op, x, B, A, D, reps=5):
    """FP16/BF16 storage and the differentiable step, each against the plain FP32 path."""
    import torch
    res = {}

    def timed(fn):
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

    y32 = op.forward_raw(x)
    b32 = op.backprojection_raw(y32)
    for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        xh = x.to(dt)
        ms = timed(lambda: op.backprojection_raw(op.forward_raw(xh)))
        yh = op.forward_raw(xh)
        bh = op.backprojection_raw(op.forward_raw(xh, scale=1e-3)) if dt == torch.float16 else \
            op.backprojection_raw(yh)
        ref_b = b32 * 1e-3 if dt == torch.float16 else b32
        res[name] = {
            "ms_per_step": round(ms, 4), "projections_per_s": round(B * A / (ms * 1e-3), 1),
            "fwd_rel_l2_vs_f32": float((yh.float() - y32).norm() / y32.norm()),
            "bp_rel_l2_vs_f32": float((bh.float() - ref_b).norm() / ref_b.norm()),
        }
    xg = x.clone().requires_grad_(True)
    yt = op.forward_raw(x)

    def ad_step():
        xg.grad = None
        loss = (op.forward(xg) - yt).pow(2).sum()
        loss.backward()

    ms = timed(ad_step)
    res["autograd_loss_step"] = {"ms_per_step": round(ms, 4),
                                 "projections_per_s": round(B * A / (ms * 1e-3), 1)}
    return res


if __name__ == "__main__":
    main()
