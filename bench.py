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
# HBM-side bytes per launch of the FP16 contraction kernel (sep_mfma8_kernel) at this
# workload, from two rocprofv3 counter runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the
# factors a plain 256 MiB elementwise copy gives),
# profiles/kde_map_gaussian_4M_2048_fp16_traffic.txt.  Set to None whenever that kernel
# changes until the counters are taken again.
TRAFFIC_FP16 = 131.5e6


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def timed_steps(torch, fn, steps: int, warmup: int, kde=None):
    """Runs warmup untimed calls, then `steps` calls, each bracketed by HIP events
    on the current stream (the stream the library launches on).  With `kde`, every
    timed call also has the library record a second pair of events around its main
    kernel alone (kde_time_next_main_kernel).  Returns (total ms, per-step ms list,
    per-step main-kernel ms list or None)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    if kde is not None:
        for a, b in kev:  # materialise the HIP events before the timed region
            a.record(stream)
            b.record(stream)
        torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(steps):
        if kde is not None:
            kde.time_next_main_kernel(*kev[i])
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    kern = [a.elapsed_time(b) for a, b in kev] if kde is not None else None
    return ev[0].elapsed_time(ev[-1]), per, kern


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Unit roundoff of the factor formats: FP16 has 11 significant bits, BF16 8.
UNIT_ROUNDOFF = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


def cpu_baseline(XY, y_maps, og, budget_s: float):
    """The FP64 oracle on the host cores over a bounded pixel sample of the same
    workload (all 4M points per pixel), on every core and on one; the GPU maps'
    errors there; and the rounding-error model of the single-pass matrix-core
    maps on the peak crop."""
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
    threads = oracle.num_threads()
    # one core: the peak 7 x 7 neighbourhood
    oracle.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.map_units_at(XY, oracle.GAUSSIAN, Hx, Hy, np.array(pix, dtype=np.int32))
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(threads)
    errs = {}
    for name, y in y_maps.items():
        yy = y[ij[:, 1], ij[:, 0]].astype(np.float64)
        errs[name] = float(np.max(np.abs(yy - r)) / np.max(np.abs(r)))
    # relative L2 on a 64 x 64 crop at the peak, separable oracle
    i0, j0 = int(min(max(ip - 32, 0), SIDE - 64)), int(min(max(jp - 32, 0), SIDE - 64))
    win = (i0, i0 + 64, j0, j0 + 64)
    raw = oracle.map_units_separable(XY, oracle.GAUSSIAN, Hx, Hy, win)
    rc = raw * scale
    crop = {}
    for name, y in y_maps.items():
        e = oracle.errors(y[win[2]:win[3], win[0]:win[1]], rc)
        crop[name] = {"e_2": e["e_2"], "e_inf": e["e_inf"]}
    # Rounding model of the single-pass paths: each factor rounded to nearest
    # carries an independent relative error of RMS u/sqrt(3), a pair product
    # u sqrt(2/3); a pixel's error then has RMS u sqrt(2/3) sqrt(sum_p w_p^2)
    # against its sum S = sum_p w_p (w_p = k(s) k(t)), i.e. relative
    # u sqrt(2/3) / sqrt(n_eff) with n_eff = S^2 / sum_p w_p^2.  For the
    # Gaussian, w_p^2 = k(s') k(t') / (2 pi) with s' = s sqrt(2): the raw map at
    # bandwidth H / sqrt(2).
    w2 = oracle.map_units_separable(XY, oracle.GAUSSIAN, np.float32(Hx / np.sqrt(2.0)),
                                    np.float32(Hy / np.sqrt(2.0)), win) / (2.0 * np.pi)
    n_eff = raw * raw / w2
    model = {"n_eff_median": float(np.median(n_eff)), "n_eff_min": float(n_eff.min())}
    for name, u in UNIT_ROUNDOFF.items():
        pred = u * np.sqrt(2.0 / 3.0) * np.sqrt(w2.sum()) / np.linalg.norm(raw)
        model[name] = {"predicted_e_2": float(pred), "measured_e_2": crop[name]["e_2"],
                       "measured_over_predicted": crop[name]["e_2"] / float(pred)}
    base = {"value": pairs / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"FP64 direct sum over all {XY.shape[0]} points at {ij.shape[0]} pixels "
                      f"(peak 7x7 neighbourhood + random), {dt:.1f} s",
            "one_core": {"value": len(pix) * XY.shape[0] / dt1, "cores": 1,
                         "sample": f"the peak 7x7 neighbourhood ({len(pix)} pixels x {XY.shape[0]} points), "
                                   f"{dt1:.1f} s"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "host_cpus_usable": len(os.sched_getaffinity(0))}
    return base, errs, crop, win, model


def transfers(torch, XY, out, map_fn, map_ms: float, pairs: float, reps: int = 5):
    """Host <-> device copies around one map, the paper's speed-up convention
    (both transfers counted): the points up (FP32 grid units, from pinned and
    from pageable host memory) and the map down (into pinned memory), each the
    median of `reps` timed copies on the current stream; end-to-end = upload
    from pinned memory + map + download."""
    import numpy as np
    stream = torch.cuda.current_stream()
    dev_pts = torch.empty(XY.shape, dtype=torch.float32, device=out.device)
    pinned = torch.from_numpy(XY).pin_memory()
    pageable = torch.from_numpy(np.ascontiguousarray(XY))
    host_map = torch.empty(out.shape, dtype=torch.float32).pin_memory()

    def timed(fn):
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return statistics.median(ms)

    up_pinned = timed(lambda: dev_pts.copy_(pinned, non_blocking=True))
    up_pageable = timed(lambda: dev_pts.copy_(pageable))
    down = timed(lambda: host_map.copy_(out, non_blocking=True))
    e2e = up_pinned + map_ms + down
    return {"points_bytes": int(XY.nbytes), "map_bytes": int(out.numel() * 4), "h2d_pinned_ms": up_pinned,
            "h2d_pageable_ms": up_pageable, "d2h_pinned_ms": down, "map_ms": map_ms, "end_to_end_ms": e2e,
            "end_to_end_pairs_per_s": pairs / (e2e * 1e-3)}


def lscv_support_pairs(XY, Hx: float, Hy: float) -> float:
    """Ordered point pairs (p = q included) with |X_p - X_q| < 2 Hx and
    |Y_p - Y_q| < 2 Hy: the pairs whose LSCV terms can be non-zero for the
    compact kernels (the autoconvolution's support), counted on the host."""
    import numpy as np
    from scipy.spatial import cKDTree
    z = np.column_stack([XY[:, 0].astype(np.float64) / (2.0 * Hx), XY[:, 1].astype(np.float64) / (2.0 * Hy)])
    tree = cKDTree(z)
    return float(tree.count_neighbors(tree, 1.0 - 1e-9, p=np.inf))


def bench_adjoint(torch, kde, synth, steps: int):
    """Adjoint workload: 250,000 points on 512 x 512, hx = hy = 0.004 degrees: the
    map VJP for the Gaussian and the Epanechnikov (L2 loss against the map of
    the Douglas-Peucker-compressed points) and the LSCV score with its gradient
    for all eight kernels.  LSCV work: the Gaussian evaluates every ordered pair;
    the compact kernels' algorithmic work is the ordered pairs closer than 2H on
    both axes (in-support pairs), reported beside the logical n^2."""
    t = synth.workload_lanes(n_tracks=500, pts=500, seed_index=3)
    tc = synth.dp_compress(t, 50.0)
    b = synth.BOX_C2
    g = kde.Grid(b.lon0, b.lon1, b.lat0, b.lat1, 512, 512)
    XY = kde.to_grid_units(t.xy, g)
    pts = torch.from_numpy(XY).cuda()
    ptc = torch.from_numpy(kde.to_grid_units(tc.xy, g)).cuda()
    n = pts.shape[0]
    res = {"points": n, "grid": [512, 512], "h_deg": 0.004, "target_points": int(ptc.shape[0])}
    for kname in ("gaussian", "epanechnikov"):
        f = kde.eval(pts, kname, 0.004, 0.004, g)
        T = kde.eval(ptc, kname, 0.004, 0.004, g)
        gbar = (2.0 * (f - T)).contiguous()
        mfma = kname == "gaussian"  # the Gaussian VJP runs on matrix cores, with one main kernel
        tot, _, kern = timed_steps(torch, lambda: kde.backward(pts, kname, 0.004, 0.004, g, gbar, want_h=False),
                                   steps, 1, kde if mfma else None)
        ms_vjp = tot / steps
        # with the bandwidth gradient (synchronises for the two host scalars)
        t0 = time.perf_counter()
        for _ in range(steps):
            kde.backward(pts, kname, 0.004, 0.004, g, gbar)
        ms_vjp_h = (time.perf_counter() - t0) * 1e3 / steps
        ent = {"vjp_ms": ms_vjp, "vjp_pairs_per_s": n * 512 * 512 / (ms_vjp * 1e-3), "vjp_with_h_ms": ms_vjp_h}
        if mfma:
            # Two contractions (Gbar^T Gy and Gbar Gx, 2 n nx ny flop each), three
            # BF16 products each (hi/lo split).
            k_ms = sum(kern) / len(kern)
            tfl = 3 * 4.0 * n * 512 * 512 / (k_ms * 1e-3) / 1e12
            tot32, _, _ = timed_steps(torch, lambda: kde.backward(pts, kname, 0.004, 0.004, g, gbar, want_h=False,
                                                                  fp32=True), steps, 1)
            ent.update({"precision": "bf16x3", "mfma_kernel_ms": k_ms, "mfma_tflops": tfl,
                        "mfma_frac": tfl / PEAK_MFMA_TFLOPS["bf16x3"], "vjp_fp32_ms": tot32 / steps})
            log(f"adjoint {kname}: vjp {ms_vjp:.2f} ms on matrix cores (main kernel {k_ms:.2f} ms, "
                f"{tfl / PEAK_MFMA_TFLOPS['bf16x3'] * 100:.1f} % of MFMA peak), FP32 {tot32 / steps:.2f} ms")
        else:
            log(f"adjoint {kname}: vjp {ms_vjp:.2f} ms")
        res[kname] = ent
    Hx, Hy = kde.bandwidth_units(0.004, 0.004, g)
    support = lscv_support_pairs(XY, float(Hx), float(Hy))
    lscv = {"ordered_pairs": float(n) * n, "in_support_pairs": support}
    for kname in kde.KERNELS:
        kde.lscv(pts, kname, 0.004, 0.004, g)
        ms = []
        for _ in range(steps):  # each call synchronises (host scalars)
            t0 = time.perf_counter()
            kde.lscv(pts, kname, 0.004, 0.004, g)
            ms.append((time.perf_counter() - t0) * 1e3)
        m = statistics.median(ms)
        ent = {"ms": m, "logical_pairs_per_s": float(n) * n / (m * 1e-3)}
        if kname != "gaussian":
            ent["in_support_pairs_per_s"] = support / (m * 1e-3)
        lscv[kname] = ent
    res["lscv"] = lscv
    log(f"lscv ({support:.3e} of {float(n) * n:.3e} ordered pairs within 2H): " +
        ", ".join(f"{k} {v['ms']:.2f} ms" for k, v in lscv.items() if isinstance(v, dict)))
    return res


def batch_window_points(torch, kde, synth, t, spec):
    """World points of one batch map: the window [start, start + count) of the
    pool, Douglas-Peucker-compressed on the GPU at the map's threshold (Mercator
    metres; 0 keeps the raw window)."""
    import numpy as np
    w = synth.window_tracks(t, spec.start, spec.count)
    if spec.eps_m == 0.0:
        return w.xy
    mx, my = synth.mercator(w.xy[:, 0], w.xy[:, 1], t.box.center_lat)
    xy = torch.from_numpy(np.column_stack([mx, my])).cuda()
    start = torch.from_numpy(np.concatenate([[0], np.cumsum(w.lengths)]).astype(np.int64)).cuda()
    keep = kde.dp_compress(xy, start, spec.eps_m, compact=False).keep.cpu().numpy().astype(bool)
    return w.xy[keep]


def batch_maps(torch, kde, synth, with_support: bool = False):
    """The 256 maps of the batch workload (see bench_batched) as kde.eval_batched
    descriptors, their specs, and (with_support) the compact maps' in-support
    pair count."""
    t = synth.workload_lanes(n_tracks=N_TRACKS, pts=PTS_PER_TRACK, seed_index=2)
    b = synth.BOX_C2
    grids = {s: kde.Grid(b.lon0, b.lon1, b.lat0, b.lat1, s, s) for s in (256, 512, 1024)}
    specs = synth.batch_specs(256, t.n)
    maps, support = [], 0.0
    for sp in specs:
        XY = kde.to_grid_units(batch_window_points(torch, kde, synth, t, sp), grids[sp.side])
        prec = "fp16" if sp.kernel == 6 else "fp32"
        maps.append((torch.from_numpy(XY).cuda(), sp.kernel, sp.h_deg, sp.h_deg, grids[sp.side],
                     torch.empty((sp.side, sp.side), device="cuda"), prec))
        if with_support and sp.kernel != 6:
            Hx, Hy = kde.bandwidth_units(sp.h_deg, sp.h_deg, grids[sp.side])
            support += map_support_pairs(XY, float(Hx), float(Hy), sp.side, sp.side)
    return maps, specs, support


def bench_batched(torch, kde, synth, steps: int):
    """Batch workload: 256 maps, each a time window of a 4M-point pool with point
    count log-uniform in [1k, 200k], Douglas-Peucker-compressed at a threshold
    drawn from {0, 10, 50, 100} m; grids from {256^2, 512^2, 1024^2}, h ~
    U(0.001, 0.008) degrees, kernels uniform over the eight.  Gaussian maps on
    the FP16 matrix-core path, the compact kernels on the FP32 persistent launch
    (graph-replayed), in one kde_eval_batched call, against 256 separate kde_eval
    launches of the same precisions.  The two parts are also timed alone."""
    maps, specs, support = batch_maps(torch, kde, synth, with_support=True)
    npts = [m[0].shape[0] for m in maps]
    pairs = float(sum(n * m[4].nx * m[4].ny for n, m in zip(npts, maps)))
    gauss = [m for m in maps if m[6] == "fp16"]
    compact = [m for m in maps if m[6] == "fp32"]
    gauss_pairs = float(sum(m[0].shape[0] * m[4].nx * m[4].ny for m in gauss))
    tot_b, _, _ = timed_steps(torch, lambda: kde.eval_batched(maps), steps, 2)
    ms_b = tot_b / steps
    tot_c, _, _ = timed_steps(torch, lambda: kde.eval_batched(compact), steps, 2)
    tot_g, _, _ = timed_steps(torch, lambda: kde.eval_batched(gauss), steps, 2)
    ms_c, ms_g = tot_c / steps, tot_g / steps

    def separate():
        for (p, k, hx, hy, g, o, prec) in maps:
            kde.eval(p, k, hx, hy, g, out=o, precision=prec)
    tot_s, _, _ = timed_steps(torch, separate, max(1, steps // 2), 1)
    ms_s = tot_s / max(1, steps // 2)
    mfma = 2.0 * gauss_pairs / (ms_g * 1e-3) / 1e12
    log(f"batched: {ms_b:.2f} ms vs separate {ms_s:.2f} ms (compact maps alone {ms_c:.2f} ms, "
        f"Gaussian maps alone {ms_g:.2f} ms = {mfma:.0f} TFLOP/s)")
    return {"maps": 256, "points_after_compression": int(sum(npts)), "points_before": int(sum(s.count for s in specs)),
            "eps_m": sorted({s.eps_m for s in specs}), "logical_pairs": pairs, "gaussian_maps": len(gauss),
            "gaussian_pairs": gauss_pairs, "compact_in_support_pairs": support,
            "batched_ms": ms_b, "separate_ms": ms_s, "batched_pairs_per_s": pairs / (ms_b * 1e-3),
            "separate_pairs_per_s": pairs / (ms_s * 1e-3), "speedup": ms_s / ms_b,
            "compact_part_ms": ms_c, "compact_in_support_pairs_per_s": support / (ms_c * 1e-3),
            "gaussian_part_ms": ms_g, "gaussian_part_mfma_tflops": mfma,
            "gaussian_part_mfma_frac": mfma / PEAK_MFMA_TFLOPS["fp16"]}


def bench_binned(torch, kde, pts, labels, g, ref_map, steps: int):
    """The paper's binned visualisation on the bench workload: count matrix with
    gap filling (one label per track), then the Eq. (7) convolution, (a) with the
    paper's 15 x 15 Gaussian table (sigma one cell) and (b) with the bench's
    bandwidth (h = 0.002 deg, taps to 6 sigma), whose map without gap filling is
    compared with the FP32 direct map (the error of the ceil binning itself)."""
    import numpy as np
    n, side = pts.shape[0], g.nx
    res = {"points": n, "grid": [side, side]}
    counts, total = kde.bin_counts(pts, labels, g)
    tot, _, _ = timed_steps(torch, lambda: kde.bin_counts(pts, labels, g, counts, total), steps, 1)
    res["counts_ms"] = tot / steps
    res["counted_cells"] = int(total.cpu().item())
    out = torch.empty((side, side), dtype=torch.float32, device=pts.device)
    H = H_DEG / g.dx
    r6 = int(np.ceil(6.0 * H))
    for name, (hx, hy, a, b) in (("paper_gauss_15x15", kde.paper_taps("gaussian", 15, g)),
                                 ("gauss_h0.002_6sigma", (H_DEG, H_DEG, r6, r6))):
        tot, _, kern = timed_steps(torch, lambda: kde.conv_counts(counts, total, "gaussian", hx, hy, a, b, g, out=out),
                                   steps, 1, kde)
        conv_ms = sum(kern) / len(kern)
        ms_full, _, _ = timed_steps(torch, lambda: kde.eval_binned(pts, labels, "gaussian", hx, hy, a, b, g, out=out),
                                    steps, 1)
        ent = {"taps": [2 * a + 1, 2 * b + 1], "conv_ms": conv_ms, "eval_binned_ms": ms_full / steps,
               "conv_hbm_gbs": 16.0 * side * side / (conv_ms * 1e-3) / 1e9,
               "logical_pairs_per_s": n * side * side / (ms_full / steps * 1e-3)}
        if name.startswith("gauss_h"):
            # without gap filling both maps are normalised by the same point count
            kde.eval_binned(pts, None, "gaussian", hx, hy, a, b, g, out=out)
            y = out.cpu().numpy().astype(np.float64)
            r = ref_map.astype(np.float64)
            peak = np.abs(r).max()
            ent["vs_fp32_direct"] = {"e_inf": float(np.abs(y - r).max() / peak),
                                     "e_2": float(np.linalg.norm(y - r) / np.linalg.norm(r))}
        res[name] = ent
    log("binned: counts %.3f ms, " % res["counts_ms"] + ", ".join(
        f"{k} conv {v['conv_ms']:.3f} ms / map {v['eval_binned_ms']:.3f} ms" for k, v in res.items()
        if isinstance(v, dict)))
    return res


def bench_truncated(torch, kde, pts, g, ref_maps, steps: int):
    """The Gaussian truncated at 8 bandwidths (KDE_TRUNCATE) on the bench
    workload: the FP32 direct path through support binning and the matrix-core
    paths banded (points binned by 256 x 256 tile), each against the full map of
    the same path.  Every dropped pair is below e^-32 of the peak pair value."""
    import numpy as np
    n, side = pts.shape[0], g.nx
    out = torch.empty((side, side), dtype=torch.float32, device=pts.device)
    res = {}
    for prec in ("fp32", "fp16", "bf16x3"):
        f = lambda: kde.eval(pts, "gaussian", H_DEG, H_DEG, g, out=out, precision=prec, truncate=True)  # noqa: E731
        tot, _, kern = timed_steps(torch, f, steps, 2, kde)
        ms = tot / steps
        y = out.cpu().numpy().astype(np.float64)
        r = ref_maps[prec].astype(np.float64)
        res[prec] = {"ms_per_map": ms, "main_kernel_ms": sum(kern) / len(kern),
                     "logical_pairs_per_s": n * side * side / (ms * 1e-3),
                     "vs_full_map_same_path": {"e_inf": float(np.abs(y - r).max() / np.abs(r).max()),
                                               "e_2": float(np.linalg.norm(y - r) / np.linalg.norm(r))}}
    res["fp32"]["shape"] = {k: v["choice"] for k, v in kde.autotune().items() if "/gtrunc/" in k}
    log("truncated Gaussian (8 h): " + ", ".join(f"{p} {v['ms_per_map']:.3f} ms" for p, v in res.items()))
    return res


def bench_dp(torch, kde, synth, t, steps: int):
    """Douglas-Peucker compression of the bench's 8,000 tracks (4,000,000 points,
    Mercator metres resident on the GPU) at eps = 10, 50, 100 m: GPU time per
    compression (mask, compaction and per-track counts), kept points, CR."""
    import numpy as np
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = torch.from_numpy(np.column_stack([mx, my])).cuda()
    start = torch.from_numpy(np.concatenate([[0], np.cumsum(t.lengths)]).astype(np.int64)).cuda()
    res = {"points": int(t.n), "tracks": int(len(t.lengths))}
    for eps in (10.0, 50.0, 100.0):
        tot, _, _ = timed_steps(torch, lambda: kde.dp_compress(xy, start, eps), steps, 1)
        keep, out, _, _ = kde.dp_compress(xy, start, eps)
        kept = int(out.shape[0])
        res[f"eps_{eps:g}m"] = {"ms": tot / steps, "points_per_s": t.n / (tot / steps * 1e-3), "kept": kept,
                                "cr_percent": (1.0 - kept / t.n) * 100.0}
    log("dp: " + ", ".join(f"{k} {v['ms']:.2f} ms (CR {v['cr_percent']:.1f} %)" for k, v in res.items()
                           if isinstance(v, dict)))
    return res


def dp_cpu_baseline(synth, t, eps: float = 50.0):
    """The oracle's sequential Douglas-Peucker on the same tracks (one core)."""
    import numpy as np

    import oracle
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = np.column_stack([mx, my])
    t0 = time.perf_counter()
    keep = oracle.dp_keep(xy, t.lengths, eps)
    dt = time.perf_counter() - t0
    return {"eps_m": eps, "ms": dt * 1e3, "points_per_s": t.n / dt, "cores": 1, "kind": "oracle",
            "kept": int(keep.sum())}


DTW_OPS_PER_CELL = 8  # FP64: 2 differences, 2 squares, 1 add (the distance), 2 min, 1 add
PEAK_FP64_OPS = 256 * 64 * 2.4e9  # FP64 VALU lane-operations per second (78.6 TFLOP/s counts an FMA twice)


def bench_metrics(torch, kde, synth, t, steps: int):
    """Compression quality of the bench's 8,000 tracks against their GPU
    Douglas-Peucker output at eps = 10, 50, 100 m (the workflow of Table IV):
    CR, RLL, DTW mean and population std.  Times the whole call and the
    per-track length + DTW kernel alone; the DTW work is the sum over tracks of
    N_o x N_c accumulated-cost cells, 8 FP64 operations each."""
    import numpy as np
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = torch.from_numpy(np.column_stack([mx, my])).cuda()
    start = torch.from_numpy(np.concatenate([[0], np.cumsum(t.lengths)]).astype(np.int64)).cuda()
    res = {"points": int(t.n), "tracks": int(len(t.lengths))}
    for eps in (10.0, 50.0, 100.0):
        _, out, lens, cst = kde.dp_compress(xy, start, eps)
        cells = float(np.sum(t.lengths.astype(np.float64) * lens.cpu().numpy().astype(np.float64)))
        tot, _, kern = timed_steps(torch, lambda: kde.compression_metrics(xy, start, out, cst, per_track=False),
                                   steps, 1, kde)
        r = kde.compression_metrics(xy, start, out, cst, per_track=False)
        k_ms = sum(kern) / len(kern)
        ops = cells * DTW_OPS_PER_CELL / (k_ms * 1e-3)
        res[f"eps_{eps:g}m"] = {"ms": tot / steps, "kernel_ms": k_ms, "dtw_cells": cells,
                                "cells_per_s": cells / (k_ms * 1e-3), "fp64_ops_per_s": ops,
                                "alu_frac": ops / PEAK_FP64_OPS, "cr_percent": r["cr_percent"], "rll": r["rll"],
                                "dtw_mean": r["dtw_mean"], "dtw_std": r["dtw_std"]}
    log("metrics: " + ", ".join(f"{k} {v['ms']:.3f} ms (kernel {v['kernel_ms']:.3f} ms, "
                                f"{v['alu_frac'] * 100:.1f} % of FP64 issue; DTW {v['dtw_mean']:.2f} +- "
                                f"{v['dtw_std']:.2f} m)" for k, v in res.items() if isinstance(v, dict)))
    return res


def metrics_cpu_baseline(synth, t, eps: float = 50.0):
    """The oracle's metrics (per-track lengths and DTW, OpenMP over tracks) on
    the same tracks against the oracle's Douglas-Peucker output."""
    import numpy as np

    import oracle
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = np.column_stack([mx, my])
    keep = oracle.dp_keep(xy, t.lengths, eps).astype(bool)
    lc = np.add.reduceat(keep.astype(np.int64), np.concatenate([[0], np.cumsum(t.lengths)[:-1]]))
    t0 = time.perf_counter()
    r = oracle.track_metrics(xy, t.lengths, xy[keep], lc)
    dt = time.perf_counter() - t0
    cells = float(np.sum(t.lengths.astype(np.float64) * lc))
    return {"eps_m": eps, "ms": dt * 1e3, "cells_per_s": cells / dt, "cores": oracle.num_threads(),
            "kind": "oracle", "dtw_mean": r["dtw_mean"]}


def map_support_pairs(XY, Hx: float, Hy: float, nx: int, ny: int) -> float:
    """(node, point) pairs with |i - X| <= Hx and |j - Y| <= Hy on the grid: the
    pairs a compact kernel's map evaluates (exact in FP64 from the FP32 inputs)."""
    import numpy as np
    X, Y = XY[:, 0].astype(np.float64), XY[:, 1].astype(np.float64)
    cx = np.clip(np.minimum(nx - 1, np.floor(X + Hx)) - np.maximum(0, np.ceil(X - Hx)) + 1, 0, None)
    cy = np.clip(np.minimum(ny - 1, np.floor(Y + Hy)) - np.maximum(0, np.ceil(Y - Hy)) + 1, 0, None)
    return float(np.sum(cx * cy))


def bench_compact(torch, kde, synth, steps: int):
    """The eight kernels on the FP32 direct path: 1,000,000 points (2,000 tracks x
    500) on 1024 x 1024, h = 0.002 degrees, raw and Douglas-Peucker-compressed at
    eps = 10, 50, 100 m (compressed on the GPU, the kept points' grid units then
    evaluated like the raw ones)."""
    import numpy as np
    t = synth.workload_lanes(n_tracks=2000, pts=500, seed_index=1)
    b = synth.BOX_C2
    g = kde.Grid(b.lon0, b.lon1, b.lat0, b.lat1, 1024, 1024)
    out = torch.empty((1024, 1024), device="cuda")
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy_m = torch.from_numpy(np.column_stack([mx, my])).cuda()
    start = torch.from_numpy(np.concatenate([[0], np.cumsum(t.lengths)]).astype(np.int64)).cuda()
    inputs = {"raw": t.xy}
    for eps in (10.0, 50.0, 100.0):
        keep = kde.dp_compress(xy_m, start, eps, compact=False).keep.cpu().numpy().astype(bool)
        inputs[f"dp_{eps:g}m"] = t.xy[keep]
    res = {}
    Hx, Hy = kde.bandwidth_units(0.002, 0.002, g)
    for name, xy in inputs.items():
        XY = kde.to_grid_units(xy, g)
        pts = torch.from_numpy(XY).cuda()
        support = map_support_pairs(XY, float(Hx), float(Hy), 1024, 1024)
        ent = {"points": int(pts.shape[0]), "in_support_pairs": support}
        for kname, kid in kde.KERNELS.items():
            tot, _, _ = timed_steps(torch, lambda: kde.eval(pts, kid, 0.002, 0.002, g, out=out), steps, 1)
            ms = tot / steps
            ent[kname] = {"ms": ms, "logical_pairs_per_s": pts.shape[0] * 1024 * 1024 / (ms * 1e-3)}
            if kname != "gaussian":
                ent[kname]["in_support_pairs_per_s"] = support / (ms * 1e-3)
        res[name] = ent
        log(f"kernels ({name}, {ent['points']} points): " + ", ".join(
            f"{k} {v['ms']:.2f} ms" for k, v in ent.items() if isinstance(v, dict)))
    return res


def calibration_copy(torch, dev) -> int:
    """A plain elementwise copy of 2^26 floats: the HBM byte counters of a
    kernel that reads and writes 256 MiB each."""
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    return src.numel() * 4


def profile_compact(torch, kde, synth) -> int:
    """Counter run for the support-binned FP32 maps: the 10^6-point workload of
    bench_compact (raw points), two maps each of the uniform, Epanechnikov and
    cosine kernels, then the calibration copy."""
    t = synth.workload_lanes(n_tracks=2000, pts=500, seed_index=1)
    b = synth.BOX_C2
    g = kde.Grid(b.lon0, b.lon1, b.lat0, b.lat1, 1024, 1024)
    out = torch.empty((1024, 1024), device="cuda")
    pts = torch.from_numpy(kde.to_grid_units(t.xy, g)).cuda()
    for kname in ("uniform", "epanechnikov", "cosine"):
        for _ in range(2):
            kde.eval(pts, kname, 0.002, 0.002, g, out=out)
    torch.cuda.synchronize()
    nb = calibration_copy(torch, out.device)
    log(f"profile run: 2 maps each of uniform, epanechnikov, cosine ({pts.shape[0]} points, 1024x1024), "
        f"then a copy of {nb} bytes read + written")
    return 0


def profile_batch(torch, kde, synth) -> int:
    """Counter run for the batch: the 256-map batch of bench_batched three
    times (the first tunes its tile sides and captures its graph), then the
    calibration copy."""
    maps, _, _ = batch_maps(torch, kde, synth)
    for _ in range(3):
        kde.eval_batched(maps)
    torch.cuda.synchronize()
    nb = calibration_copy(torch, torch.device("cuda:0"))
    log(f"profile run: 3 calls of the 256-map batch, then a copy of {nb} bytes read + written")
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--direct-steps", type=int, default=3, help="timed steps of the FP32 direct path")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-once", nargs="?", const="headline", choices=("headline", "compact", "batch"),
                    help="for counter runs, prints no JSON: 'headline' (the default) runs two FP16 maps and one "
                         "FP32 direct map of the 4M-point workload, 'compact' two uniform, Epanechnikov and "
                         "cosine maps each of 10^6 points on 1024 x 1024, 'batch' three calls of the 256-map "
                         "batch; then a 256 MiB elementwise copy (torch.neg) as the byte-count calibration")
    ap.add_argument("--sections", default="adjoint,batched,kernels,binned,truncated,dp,metrics",
                    help="extra measured sections beside the headline: adjoint, batched, kernels, binned, "
                         "truncated, dp, metrics (or none)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the KDE map runs on a single MI355X here "
              "(sharding the map across GPUs is not built in this library).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2004_13653_amd as kde
    import synth

    if args.profile_once == "compact":
        return profile_compact(torch, kde, synth)
    if args.profile_once == "batch":
        return profile_batch(torch, kde, synth)
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

    if args.profile_once:
        f = run("fp16")
        f()
        f()
        run("fp32")()
        nb = calibration_copy(torch, dev)
        log(f"profile run: 2 FP16 maps, 1 FP32 direct map, then a copy of {nb} bytes read + written")
        return 0

    results, maps = {}, {}
    for prec in ("fp16", "bf16", "fp16x3", "bf16x3", "fp32"):
        steps = args.steps if prec != "fp32" else args.direct_steps
        warm = args.warmup if prec != "fp32" else 1
        total, per, kern = timed_steps(torch, run(prec), steps, warm, kde)
        ms = total / steps
        results[prec] = {"ms_per_step": ms, "median_ms": statistics.median(per), "value": pairs / (ms * 1e-3),
                         "steps": steps, "main_kernel_ms": sum(kern) / len(kern)}
        maps[prec] = out.cpu().numpy().copy()
        log(f"{prec}: {ms:.3f} ms/step  {pairs / (ms * 1e-3):.3e} pairs/s")

    head = results["fp16"]
    line_transfers = transfers(torch, XY, out, run("fp16"), head["ms_per_step"], pairs)
    mult = {"fp16": 1, "bf16": 1, "fp16x3": 3, "bf16x3": 3}
    for prec in mult:
        tfl = 2.0 * mult[prec] * pairs / (results[prec]["main_kernel_ms"] * 1e-3) / 1e12
        results[prec]["mfma_tflops"] = tfl
        results[prec]["mfma_frac"] = tfl / PEAK_MFMA_TFLOPS[prec]
    d = results["fp32"]
    d["fp32_tflops"] = 2.0 * pairs / (d["main_kernel_ms"] * 1e-3) / 1e12

    # Algorithmic work of one launch of the contraction kernel: 2 flop per
    # pixel x point pair (one multiply-add of the rank-n product Gy Gx^T).
    achieved = 2.0 * pairs / (head["main_kernel_ms"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_TFLOPS["fp16"], "unit": "TFLOP/s",
                "frac": achieved / PEAK_MFMA_TFLOPS["fp16"], "traffic": TRAFFIC_FP16,
                "kernel": "sep_mfma8_kernel<fp16> (dense Gaussian runs)", "kernel_ms": head["main_kernel_ms"],
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
        "transfers": line_transfers,
    }
    extra = [x for x in args.sections.split(",") if x and x != "none"]
    if "adjoint" in extra:
        line["adjoint"] = bench_adjoint(torch, kde, synth, 5)
    if "batched" in extra:
        line["batched"] = bench_batched(torch, kde, synth, 6)
    if "kernels" in extra:
        line["fp32_direct_kernels"] = bench_compact(torch, kde, synth, 5)
    if "dp" in extra:
        line["dp"] = bench_dp(torch, kde, synth, t, 5)
    if "metrics" in extra:
        line["metrics"] = bench_metrics(torch, kde, synth, t, 5)
    if "truncated" in extra:
        line["truncated"] = bench_truncated(torch, kde, pts, g, maps, 10)
    if "binned" in extra:
        lab = torch.from_numpy(np.repeat(np.arange(len(t.lengths), dtype=np.int32), t.lengths)).to(dev)
        line["binned"] = bench_binned(torch, kde, pts, lab, g, maps["fp32"], 10)
    if not args.no_cpu_baseline:
        og_mod = __import__("oracle")
        og = og_mod.Grid(b.lon0, b.lon1, b.lat0, b.lat1, SIDE, SIDE)
        base, errs, crop, win, model = cpu_baseline(XY, maps, og, args.cpu_budget)
        line["cpu_baseline"] = base
        line["mfma_error_model"] = model
        if "dp" in extra:
            line["dp"]["cpu_baseline"] = dp_cpu_baseline(synth, t)
            line["dp"]["speedup_vs_cpu_eps_50m"] = line["dp"]["cpu_baseline"]["ms"] / line["dp"]["eps_50m"]["ms"]
        if "metrics" in extra:
            line["metrics"]["cpu_baseline"] = metrics_cpu_baseline(synth, t)
            line["metrics"]["speedup_vs_cpu_eps_50m"] = (line["metrics"]["cpu_baseline"]["ms"]
                                                        / line["metrics"]["eps_50m"]["ms"])
        line["error_vs_fp64"] = {"sampled_e_inf": errs, "peak_crop": {"window": list(win), **crop}}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
