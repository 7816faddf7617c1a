"""Batched persistent launch (kde_eval_batched) against separate kde_eval calls
and the FP64 oracle, eager and graph-replayed."""
import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt

pytestmark = pytest.mark.gpu


def _batch(specs, pool_units_by_side, grids):
    """(points tensor, kernel, hx, hy, grid, out tensor) per spec."""
    import torch
    maps = []
    for s in specs:
        XY = pool_units_by_side[s.side][s.start:s.start + s.count]
        pts = kt.to_device(XY) if s.count else torch.empty((0, 2), device=kt.device())
        out = torch.full((s.side, s.side), float("nan"), device=kt.device())
        maps.append((pts, s.kernel, s.h_deg, s.h_deg, grids[s.side], out))
    return maps


def _pool(n_tracks):
    t = kt.lanes(n_tracks, 500, 3)
    b = synth.BOX_C2
    grids = {s: kde.Grid(b.lon0, b.lon1, b.lat0, b.lat1, s, s) for s in (64, 100, 256, 512, 1024)}
    units = {s: kde.to_grid_units(t.xy, g) for s, g in grids.items()}
    return t, grids, units


@pytest.mark.parametrize("eager", [True, False])
def test_small_mixed_batch_matches_separate_and_oracle(eager):
    import torch
    t, grids, units = _pool(100)
    specs = [synth.MapSpec(0, 0, 64, 0.01, 6),            # empty
             synth.MapSpec(5, 1, 100, 0.02, 0),            # one point
             synth.MapSpec(100, 20000, 256, 0.004, 6),     # Gaussian, split into point ranges
             synth.MapSpec(3000, 7000, 100, 0.015, 6),     # Gaussian, ragged 100 x 100 grid
             synth.MapSpec(0, 30000, 256, 0.003, 2)]
    specs += [synth.MapSpec(1000 * k, 4000 + 500 * k, (64, 100, 256)[k % 3], 0.003 + 0.002 * k, k) for k in range(8)]
    maps = _batch(specs, units, grids)
    kde.eval_batched(maps, eager=eager)
    torch.cuda.synchronize()
    for s, (pts, kernel, hx, hy, g, out) in zip(specs, maps):
        y = out.cpu().numpy().astype(np.float64)
        ref = kde.eval(pts, kernel, hx, hy, g) if s.count else torch.zeros_like(out)
        torch.cuda.synchronize()
        r = ref.cpu().numpy().astype(np.float64)
        assert np.isfinite(y).all()
        if s.count == 0:
            assert np.all(y == 0.0)
            continue
        assert kt.peak_error(y, r) <= 2e-6, s
        og = oracle.Grid(*g.bounds, g.nx, g.ny)
        ro = kt.oracle_density_window(units[s.side][s.start:s.start + s.count], kernel, hx, hy, og,
                                      (0, g.nx, 0, g.ny), separable=True)
        assert kt.peak_error(y, ro) <= kt.FP32_GATE, s


@pytest.mark.parametrize("eager", [True, False])
def test_small_support_compact_maps_equal_kde_eval_bit_for_bit(eager):
    """Compact maps whose supports span at most 225 tried nodes (441 for the
    cosine) sum in 64-bit fixed point in both paths (support-binned items in kde_eval, chunk-box tiles in the
    batch), so the maps agree bit for bit whatever tile sides the two take: the
    batch with 32-, 64- and 128-node tiles against kde_eval with 32-node tiles.
    The 64 x 64 map puts about 5000 points in each tile, which kde_eval cuts into
    several items; one map is anisotropic and two sit at the footprint limits."""
    import math
    import torch
    t, grids, units = _pool(100)
    units[1024] = kde.to_grid_units(t.xy, grids[1024])
    rows = [(0, 20000, 64, 0.02, 0.02, 0), (5000, 12000, 100, 0.01, 0.01, 2), (0, 30000, 256, 0.005, 0.005, 7),
            (10000, 25000, 512, 0.003, 0.003, 5), (20000, 30000, 1024, 0.006, 0.006, 4),
            (3000, 9000, 512, 0.004, 0.002, 1), (40000, 8000, 256, 0.006, 0.006, 3),
            (0, 20000, 1024, 0.009, 0.009, 7)]
    for (_, _, side, hx, hy, k) in rows:  # every map takes the fixed-point path, two at its limits
        Hx, Hy = kde.bandwidth_units(hx, hy, grids[side])
        assert (math.floor(2 * Hx) + 3) * (math.floor(2 * Hy) + 3) <= (441 if k == 7 else 225)
    pts = [kt.to_device(units[side][a:a + n]) for (a, n, side, _, _, _) in rows]
    try:
        kde.autotune(force=2)
        refs = [kde.eval(p, k, hx, hy, grids[side]).cpu().numpy()
                for p, (_, _, side, hx, hy, k) in zip(pts, rows)]
        for rc in (2, 4, 8):
            kde.autotune(force=rc)
            maps = [(p, k, hx, hy, grids[side], torch.full((side, side), float("nan"), device=kt.device()))
                    for p, (_, _, side, hx, hy, k) in zip(pts, rows)]
            kde.eval_batched(maps, eager=eager)
            torch.cuda.synchronize()
            for m, r, row in zip(maps, refs, rows):
                np.testing.assert_array_equal(m[5].cpu().numpy(), r, err_msg=f"tile side {16 * rc}, map {row}")
    finally:
        kde.autotune(force=0)
    a, n, side, hx, hy, k = rows[0]
    og = oracle.Grid(*grids[side].bounds, side, side)
    ro = kt.oracle_density_window(units[side][a:a + n], k, hx, hy, og, (0, side, 0, side), separable=True)
    assert kt.peak_error(refs[0].astype(np.float64), ro) <= kt.FP32_GATE


def test_graph_replays_track_new_inputs():
    """Same batch shape three times with different points and bandwidth-dependent
    scales (same grids and counts): every replay equals separate calls; eager
    torch work runs between replays."""
    import torch
    t, grids, units = _pool(100)
    base = [synth.MapSpec(0, 9000, 256, 0.004, 6), synth.MapSpec(0, 5000, 100, 0.01, 3),
            synth.MapSpec(0, 12000, 64, 0.02, 7)]
    for rep in range(3):
        specs = [synth.MapSpec(s.start + 7000 * rep, s.count, s.side, s.h_deg * (1 + 0.1 * rep), s.kernel)
                 for s in base]
        maps = _batch(specs, units, grids)
        kde.eval_batched(maps)
        junk = torch.randn(1 << 20, device=kt.device()).sum()  # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for s, (pts, kernel, hx, hy, g, out) in zip(specs, maps):
            ref = kde.eval(pts, kernel, hx, hy, g)
            torch.cuda.synchronize()
            assert kt.peak_error(out.cpu().numpy(), ref.cpu().numpy()) <= 2e-6, (rep, s)


PREC_GATE = {"fp32": ("e_inf", kt.FP32_GATE), "fp16": ("e_2", 2e-3), "bf16x3": ("e_2", 2e-3)}
# Batched matrix-core maps against kde_eval: the same products, summed over
# fewer point splits (FP32 accumulation in another order).
SPLIT_ORDER_GATE = 1e-5


def _window_points(pool, spec):
    """World points of the batch map: the window [start, start + count) of the
    pool, Douglas-Peucker-compressed (the oracle's, on Mercator metres) at the
    map's threshold; 0 keeps the raw window."""
    w = synth.window_tracks(pool, spec.start, spec.count)
    if spec.eps_m == 0.0:
        return w.xy
    mx, my = synth.mercator(w.xy[:, 0], w.xy[:, 1], pool.box.center_lat)
    keep = oracle.dp_keep(np.column_stack([mx, my]), w.lengths, spec.eps_m).astype(bool)
    return w.xy[keep]


def _c5_precision(k, spec):
    """Gaussian maps on the matrix cores (FP16, every fourth on the BF16 hi/lo
    split), the compact kernels on the FP32 persistent launch."""
    if spec.kernel != oracle.GAUSSIAN:
        return "fp32"
    return "bf16x3" if k % 4 == 0 else "fp16"


@pytest.mark.timeout(900)
def test_batch_of_256_time_windows():
    """256 maps: windows of a 4M-point pool with point counts log-uniform in
    [1k, 200k], each Douglas-Peucker-compressed at a threshold from {0, 10, 50,
    100} m, grids from {256^2, 512^2, 1024^2}, h ~ U(0.001, 0.008) degrees,
    kernels uniform over the eight; Gaussian maps on the matrix cores.  Every map
    against a separate kde_eval call of its precision (the matrix-core maps
    split their points more coarsely in the batch: equal up to the FP32 order of
    the split sums), and for every precision some maps against the oracle at
    sampled pixels, each at its precision's gate."""
    import torch
    t = kt.lanes(8000, 500, 2)
    b = synth.BOX_C2
    grids = {s: kde.Grid(b.lon0, b.lon1, b.lat0, b.lat1, s, s) for s in (256, 512, 1024)}
    ogrids = {s: oracle.Grid(b.lon0, b.lon1, b.lat0, b.lat1, s, s) for s in (256, 512, 1024)}
    specs = synth.batch_specs(256, t.n)
    assert {s.eps_m for s in specs} == {0.0, 10.0, 50.0, 100.0}
    maps, units = [], []
    for k, s in enumerate(specs):
        XY = kde.to_grid_units(_window_points(t, s), grids[s.side])
        units.append(XY)
        out = torch.full((s.side, s.side), float("nan"), device=kt.device())
        maps.append((kt.to_device(XY), s.kernel, s.h_deg, s.h_deg, grids[s.side], out, _c5_precision(k, s)))
    kt.log(f"256 windows: {sum(u.shape[0] for u in units)} points after compression "
           f"(of {sum(s.count for s in specs)}), precisions "
           f"{ {p: sum(1 for m in maps if m[6] == p) for p in PREC_GATE} }")
    kde.eval_batched(maps)
    torch.cuda.synchronize()
    worst, checked = 0.0, {p: 0 for p in PREC_GATE}
    for k, (s, (pts, kernel, hx, hy, g, out, prec)) in enumerate(zip(specs, maps)):
        ref = kde.eval(pts, kernel, hx, hy, g, precision=prec)
        torch.cuda.synchronize()
        y, r = out.cpu().numpy(), ref.cpu().numpy()
        if prec == "fp32":
            e = kt.peak_error(y, r)
            worst = max(worst, e)
            assert e <= 2e-6, (k, s)
        else:
            assert kt.peak_error(y, r) <= SPLIT_ORDER_GATE, (k, s)
        if checked[prec] < 3 and (prec != "fp32" or k % 32 == 0):
            checked[prec] += 1
            yy = y.astype(np.float64)
            ij = kt.sample_pixels(yy, 16, seed=k)
            ro = kt.oracle_density_at(units[k], kernel, hx, hy, ogrids[s.side], ij)
            e = oracle.errors(yy[ij[:, 1], ij[:, 0]], ro)
            name, gate = PREC_GATE[prec]
            kt.log(f"map {k} ({prec}, kernel {kernel}, eps {s.eps_m} m, n {units[k].shape[0]}): "
                   f"e_inf {e['e_inf']:.2e} e_2 {e['e_2']:.2e}")
            assert e[name] <= gate, (k, s)
    assert all(v >= 2 for v in checked.values()), checked
    kt.log(f"256 maps: worst peak-normalised FP32 difference to separate calls {worst:.2e}")


@pytest.mark.parametrize("eager", [True, False])
def test_mixed_precision_batch(eager):
    """FP32, matrix-core and truncated maps in one call: the persistent launch
    for the FP32 maps, the others one by one after it; each equals kde_eval of
    its precision (bit for bit for the single launches, up to the order of the
    split sums for the batched matrix-core Gaussian maps), empty maps are zero."""
    import torch
    t, grids, units = _pool(100)
    cases = [(synth.MapSpec(100, 20000, 256, 0.004, 6), "fp16", False),
             (synth.MapSpec(3000, 7000, 100, 0.015, 6), "bf16", False),
             (synth.MapSpec(0, 30000, 256, 0.003, 2), "fp16x3", False),
             (synth.MapSpec(500, 9000, 256, 0.004, 6), "fp32", True),
             (synth.MapSpec(900, 15000, 100, 0.01, 6), "bf16x3", True),
             (synth.MapSpec(0, 0, 64, 0.01, 6), "fp16", False),
             (synth.MapSpec(1000, 6000, 64, 0.02, 3), "fp32", False),
             (synth.MapSpec(2000, 8000, 256, 0.004, 6), "fp32", False)]
    maps = []
    for s, prec, trunc in cases:
        XY = units[s.side][s.start:s.start + s.count]
        pts = kt.to_device(XY) if s.count else torch.empty((0, 2), device=kt.device())
        out = torch.full((s.side, s.side), float("nan"), device=kt.device())
        maps.append((pts, s.kernel, s.h_deg, s.h_deg, grids[s.side], out, prec, trunc))
    kde.eval_batched(maps, eager=eager)
    torch.cuda.synchronize()
    for (s, prec, trunc), (pts, kernel, hx, hy, g, out, _, _) in zip(cases, maps):
        y = out.cpu().numpy()
        if s.count == 0:
            assert np.all(y == 0.0)
            continue
        ref = kde.eval(pts, kernel, hx, hy, g, precision=prec, truncate=trunc).cpu().numpy()
        if prec == "fp32" and not trunc:
            assert kt.peak_error(y, ref) <= 2e-6, (s, prec)
        elif kernel == 6 and not trunc:
            assert kt.peak_error(y, ref) <= SPLIT_ORDER_GATE, (s, prec)
        else:
            np.testing.assert_array_equal(y, ref)


@pytest.mark.parametrize("eager", [True, False])
def test_dense_gaussian_maps_share_one_launch(eager):
    """The Gaussian maps of each matrix-core precision go out as one launch of
    the contraction kernel with multiplicative runs, and those too narrow for
    runs as one launch of the kernel that evaluates every factor (plus one
    padding and one split-reduction launch each): maps of one and of several
    point splits, one to sixteen 256-node tiles, ragged grids.  Each map equals
    kde_eval up to the order of the split sums, and sampled maps match the
    oracle at their precision's gate."""
    import torch
    t, grids, units = _pool(100)
    cases = []
    for prec in ("fp16", "bf16", "fp16x3", "bf16x3"):
        cases += [(synth.MapSpec(0, 45000, 512, 0.003, 6), prec),    # four tiles, several splits
                  (synth.MapSpec(2000, 300, 100, 0.02, 6), prec),    # one ragged tile, one split
                  (synth.MapSpec(7000, 9000, 1024, 0.002, 6), prec),  # sixteen tiles
                  (synth.MapSpec(100, 5000, 256, 0.0004, 6), prec)]  # H < 1.05 px: no runs, the other kernel
    maps = []
    for s, prec in cases:
        XY = units[s.side][s.start:s.start + s.count]
        out = torch.full((s.side, s.side), float("nan"), device=kt.device())
        maps.append((kt.to_device(XY), s.kernel, s.h_deg, s.h_deg, grids[s.side], out, prec))
    for _ in range(2):  # the second call reuses the staged table buffer
        kde.eval_batched(maps, eager=eager)
        torch.cuda.synchronize()
        for (s, prec), (pts, kernel, hx, hy, g, out, _) in zip(cases, maps):
            ref = kde.eval(pts, kernel, hx, hy, g, precision=prec).cpu().numpy()
            assert kt.peak_error(out.cpu().numpy(), ref) <= SPLIT_ORDER_GATE, (s, prec)
    og = oracle.Grid(*grids[100].bounds, 100, 100)
    for k in (1, 5, 9, 13):  # the 100 x 100 map of every precision
        s, prec = cases[k]
        r = kt.oracle_density_window(units[100][s.start:s.start + s.count], 6, s.h_deg, s.h_deg, og,
                                     (0, 100, 0, 100))
        e = oracle.errors(maps[k][5].cpu().numpy().astype(np.float64).ravel(), r.ravel())
        kt.log(f"{prec}: e_2 {e['e_2']:.2e} e_inf {e['e_inf']:.2e}")
        assert e["e_2"] <= 2e-3, (s, prec, e)
    og = oracle.Grid(*grids[256].bounds, 256, 256)
    for k in (3, 7, 11, 15):  # the narrow 256 x 256 map of every precision, at sampled pixels
        s, prec = cases[k]
        y = maps[k][5].cpu().numpy().astype(np.float64)
        ij = kt.sample_pixels(y, 64, seed=k)
        r = kt.oracle_density_at(units[256][s.start:s.start + s.count], 6, s.h_deg, s.h_deg, og, ij)
        e = oracle.errors(y[ij[:, 1], ij[:, 0]], r)
        kt.log(f"{prec} narrow: e_2 {e['e_2']:.2e} e_inf {e['e_inf']:.2e}")
        assert e["e_2"] <= 2e-3, (s, prec, e)


@pytest.mark.parametrize("rc", [2, 4, 8])
def test_forced_tile_shapes_match_oracle(rc):
    """The persistent kernel with every register-block shape forced (Gaussian
    maps then also split into point ranges of other sizes)."""
    import torch
    t, grids, units = _pool(100)
    specs = [synth.MapSpec(100, 20000, 256, 0.004, 6), synth.MapSpec(3000, 7000, 100, 0.015, 6)]
    specs += [synth.MapSpec(1000 * k, 4000 + 500 * k, (64, 100, 256)[k % 3], 0.003 + 0.002 * k, k) for k in range(8)]
    try:
        kde.autotune(force=rc)
        maps = _batch(specs, units, grids)
        kde.eval_batched(maps)
        torch.cuda.synchronize()
    finally:
        kde.autotune(force=0)
    for s, (pts, kernel, hx, hy, g, out) in zip(specs, maps):
        y = out.cpu().numpy().astype(np.float64)
        og = oracle.Grid(*g.bounds, g.nx, g.ny)
        ro = kt.oracle_density_window(units[s.side][s.start:s.start + s.count], kernel, hx, hy, og,
                                      (0, g.nx, 0, g.ny), separable=True)
        assert kt.peak_error(y, ro) <= kt.FP32_GATE, (rc, s)


def test_batch_shapes_are_tuned_once():
    """A new batch composition is tuned (whole-batch runs per shape pair), the
    choice cached under a batch key and reused by the next call."""
    import torch
    t, grids, units = _pool(100)
    specs = [synth.MapSpec(0, 9000, 256, 0.004, 6), synth.MapSpec(0, 15000, 100, 0.01, 3),
             synth.MapSpec(500, 12000, 64, 0.02, 7), synth.MapSpec(900, 30000, 256, 0.003, 0)]
    kde.autotune(clear=True, enabled=True, force=0)
    maps = _batch(specs, units, grids)
    kde.eval_batched(maps)
    torch.cuda.synchronize()
    ent = kde.autotune()
    keys = [k for k in ent if k.startswith("batch/")]
    assert len(keys) == 1, ent
    e = ent[keys[0]]
    kt.log(f"{keys[0]}: {e}")
    assert e["choice"] in e["ms"] and e["ms"][e["choice"]] == min(e["ms"].values())
    first = [m[5].cpu().numpy() for m in maps]
    kde.eval_batched(maps)
    torch.cuda.synchronize()
    assert kde.autotune() == ent
    for a, m in zip(first, maps):
        np.testing.assert_array_equal(a, m[5].cpu().numpy())


@pytest.mark.parametrize("eager", [True, False])
def test_non_finite_points_contribute_nothing_to_compact_maps(eager):
    """Points with NaN or infinite coordinates add nothing to a compact map, as
    kde_eval's contract states: with raw sums (no 1/n), the map of a point set
    laced with them equals the map of its finite points, single and batched, on
    the fixed-point path (small supports), the binned gather (large supports)
    and the unbinned sums (n < 4096, and the batch's gather).  Bit for bit on
    the fixed-point path, whose sums do not depend on order or grouping;
    elsewhere the inserted points shift the 64-point scatter groups and the
    256-point chunks, so the FP32 partial sums associate differently."""
    import torch
    t, grids, units = _pool(100)
    rng = np.random.default_rng(17)
    bad_vals = [np.nan, np.inf, -np.inf]
    # (start, count, side, h, kernel, exact single, exact batched)
    rows = [(0, 20000, 256, 0.005, 0, True, True),       # fixed point both ways (H = 1.3)
            (3000, 12000, 512, 0.003, 7, True, True),    # fixed point both ways (H = 1.5)
            (0, 20000, 256, 0.03, 7, False, False),      # binned gather; chunk-box gather (H = 7.7)
            (5000, 9000, 100, 0.05, 3, False, False),    # the same on a ragged grid (H = 5.0)
            (100, 3000, 256, 0.005, 2, False, True)]     # unbinned single map; fixed point batched
    finite, laced = [], []
    for (a, n, side, h, k, _, _) in rows:
        XY = units[side][a:a + n].astype(np.float32)
        bad = np.empty((n // 50, 2), np.float32)
        for r in range(bad.shape[0]):  # one or both coordinates non-finite, the other in the grid
            bad[r] = XY[rng.integers(0, n)]
            which = rng.integers(0, 3)
            if which != 1:
                bad[r, 0] = bad_vals[rng.integers(0, 3)]
            if which != 0:
                bad[r, 1] = bad_vals[rng.integers(0, 3)]
        mixed = np.insert(XY, rng.integers(0, n, bad.shape[0]), bad, axis=0)
        finite.append(kt.to_device(XY))
        laced.append(kt.to_device(mixed))
    def same(got, ref, exact, what):
        assert np.isfinite(got).all(), what
        if exact:
            np.testing.assert_array_equal(got, ref, err_msg=what)
        else:
            assert kt.peak_error(got, ref) <= 1e-6, what
    for row, pf, pl in zip(rows, finite, laced):
        a, n, side, h, k, exact, _ = row
        ref = kde.eval(pf, k, h, h, grids[side], raw=True).cpu().numpy()
        got = kde.eval(pl, k, h, h, grids[side], raw=True).cpu().numpy()
        same(got, ref, exact, f"kde_eval {row}")
    for pts in (finite, laced):
        maps = [(p, k, h, h, grids[side], torch.full((side, side), float("nan"), device=kt.device()))
                for p, (a, n, side, h, k, _, _) in zip(pts, rows)]
        kde.eval_batched(maps, raw=True, eager=eager)
        torch.cuda.synchronize()
        if pts is finite:
            ref_b = [m[5].cpu().numpy() for m in maps]
        else:
            for m, r, row in zip(maps, ref_b, rows):
                same(m[5].cpu().numpy(), r, row[6], f"kde_eval_batched {row}")
