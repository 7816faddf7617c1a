"""Benchmark: KDE heat map, matrix-core separable path against the FP32 direct
kernel, on one MI355X.

Workload: 4,000,000 synthetic AIS points (8,000 vessel tracks x 500 reports,
crossing lanes plus anchored clusters, 1 x 1 degree box) on a 2048 x 2048 grid,
Gaussian kernel, hx = hy = 0.002 degrees; points resident in HBM as FP32 grid
units before timing starts.  One step = one full map (kde_eval) on the FP16
separable path.  The FP32 direct path, BF16 and the hi/lo splits are timed on
the same input beside it.  Metric: pixel x point evaluations per second.

Prints one JSON line (see the fields at the end of main()).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pixel×point evals/s: MFMA separable vs FP32 direct KDE at stated error"
UNIT = "pixel×point evals/s"
PEAK_MFMA_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp16x3": 2500.0, "bf16x3": 2500.0}
PEAK_FP32_VECTOR_TFLOPS = 157.3
N_TRACKS, PTS_PER_TRACK, SIDE, H_DEG = 8000, 500, 2048, 0.002


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def timed_steps(torch, fn, steps: int, warmup: int):
    """Runs warmup untimed calls, then `steps` calls, each bracketed by HIP events
    on the current stream (the stream the library launches on).  Returns
    (total ms, per-step ms list)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[-1]), per


def cpu_baseline(XY, y_maps, og, budget_s: float):
    """The FP64 oracle on the host cores over a bounded pixel sample of the same
    workload (all 4M points per pixel), plus the GPU maps' errors there."""
    import numpy as np

    import oracle
    Hx, Hy = oracle.bandwidth_units(H_DEG, H_DEG, og)
    scale = oracle.density_scale(XY.shape[0], H_DEG, H_DEG)
    ref_map = y_maps["fp32"]
    jp, ip = np.unravel_index(np.argmax(ref_map), ref_map.shape)
    rng = np.random.default_rng(2004)
    pix = [(int(ip + di), int(jp + dj)) for dj in range(-3, 4) for di in range(-3, 4)
           if 0 <= ip + di < SIDE and 0 <= jp + dj < SIDE]
    done_ij, vals = [], []
    t0 = time.perf_counter()
    batch = list(pix)
    while True:
        ij = np.array(batch, dtype=np.int32)
        vals.append(oracle.map_units_at(XY, oracle.GAUSSIAN, Hx, Hy, ij) * scale)
        done_ij.append(ij)
        if time.perf_counter() - t0 > budget_s:
            break
        batch = [(int(rng.integers(0, SIDE)), int(rng.integers(0, SIDE))) for _ in range(64)]
    dt = time.perf_counter() - t0
    ij = np.concatenate(done_ij)
    r = np.concatenate(vals)
    pairs = ij.shape[0] * XY.shape[0]
    errs = {}
    for name, y in y_maps.items():
        yy = y[ij[:, 1], ij[:, 0]].astype(np.float64)
        errs[name] = float(np.max(np.abs(yy - r)) / np.max(np.abs(r)))
    # relative L2 on a 64 x 64 crop at the peak, separable oracle
    i0, j0 = int(min(max(ip - 32, 0), SIDE - 64)), int(min(max(jp - 32, 0), SIDE - 64))
    win = (i0, i0 + 64, j0, j0 + 64)
    rc = oracle.map_units_separable(XY, oracle.GAUSSIAN, Hx, Hy, win) * scale
    crop = {}
    for name, y in y_maps.items():
        e = oracle.errors(y[win[2]:win[3], win[0]:win[1]], rc)
        crop[name] = {"e_2": e["e_2"], "e_inf": e["e_inf"]}
    base = {"value": pairs / dt, "unit": UNIT, "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 direct sum over all {XY.shape[0]} points at {ij.shape[0]} pixels "
                      f"(peak 7x7 neighbourhood + random), {dt:.1f} s"}
    return base, errs, crop, win


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--direct-steps", type=int, default=3, help="timed steps of the FP32 direct path")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the KDE map runs on a single MI355X here "
              "(sharding the map across GPUs is not built in this library).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2004_13653_amd as kde
    import synth

    t = synth.workload_lanes(n_tracks=N_TRACKS, pts=PTS_PER_TRACK, seed_index=2)
    b = synth.BOX_C2
    g = kde.Grid(b.lon0, b.lon1, b.lat0, b.lat1, SIDE, SIDE)
    XY = kde.to_grid_units(t.xy, g)
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(XY).to(dev)
    out = torch.empty((SIDE, SIDE), dtype=torch.float32, device=dev)
    n = XY.shape[0]
    pairs = n * SIDE * SIDE
    log(f"workload: n={n} grid={SIDE}x{SIDE} gaussian h={H_DEG} deg")

    def run(prec):
        return lambda: kde.eval(pts, "gaussian", H_DEG, H_DEG, g, out=out, precision=prec)

    results, maps = {}, {}
    for prec in ("fp16", "bf16", "fp16x3", "bf16x3", "fp32"):
        steps = args.steps if prec != "fp32" else args.direct_steps
        warm = args.warmup if prec != "fp32" else 1
        total, per = timed_steps(torch, run(prec), steps, warm)
        ms = total / steps
        results[prec] = {"ms_per_step": ms, "median_ms": statistics.median(per), "value": pairs / (ms * 1e-3),
                         "steps": steps}
        maps[prec] = out.cpu().numpy().copy()
        log(f"{prec}: {ms:.3f} ms/step  {pairs / (ms * 1e-3):.3e} pairs/s")

    head = results["fp16"]
    mult = {"fp16": 1, "bf16": 1, "fp16x3": 3, "bf16x3": 3}
    for prec in mult:
        tfl = 2.0 * mult[prec] * pairs / (results[prec]["ms_per_step"] * 1e-3) / 1e12
        results[prec]["mfma_tflops"] = tfl
        results[prec]["mfma_frac"] = tfl / PEAK_MFMA_TFLOPS[prec]
    d = results["fp32"]
    d["fp32_tflops"] = 2.0 * pairs / (d["ms_per_step"] * 1e-3) / 1e12

    achieved = 2.0 * pairs / (head["ms_per_step"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_TFLOPS["fp16"], "unit": "TFLOP/s",
                "frac": achieved / PEAK_MFMA_TFLOPS["fp16"], "traffic": None,
                "kernel": "sep_mfma_kernel<gaussian, fp16> (+ split reduction)",
                "flops_per_launch": 2.0 * pairs}

    line = {
        "metric": METRIC, "value": head["value"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp16", "data": "synthetic",
        "config": {"workload": "KDE heat map, 4M AIS-shaped points (8000 tracks x 500) on a 2048x2048 grid, "
                               "Gaussian, h=0.002 deg, FP16 separable MFMA path",
                   "points": n, "grid": [SIDE, SIDE], "kernel": "gaussian", "h_deg": H_DEG,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "speedup_vs_fp32_direct": head["value"] / d["value"],
        "fp32_direct": {"value": d["value"], "ms_per_step": d["ms_per_step"], "steps": d["steps"],
                        "roofline": {"bound": "alu", "achieved": d["fp32_tflops"], "peak": PEAK_FP32_VECTOR_TFLOPS,
                                     "unit": "TFLOP/s", "frac": d["fp32_tflops"] / PEAK_FP32_VECTOR_TFLOPS}},
        "paths": results,
    }
    if not args.no_cpu_baseline:
        og_mod = __import__("oracle")
        og = og_mod.Grid(b.lon0, b.lon1, b.lat0, b.lat1, SIDE, SIDE)
        base, errs, crop, win = cpu_baseline(XY, maps, og, args.cpu_budget)
        line["cpu_baseline"] = base
        line["error_vs_fp64"] = {"sampled_e_inf": errs, "peak_crop": {"window": list(win), **crop}}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
