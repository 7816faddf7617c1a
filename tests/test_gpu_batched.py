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


def test_batch_of_256_time_windows():
    """256 maps: point counts log-uniform in [1k, 200k] (slices of a 4M-point
    pool), grids from {256^2, 512^2, 1024^2}, h ~ U(0.001, 0.008) degrees, kernels
    uniform over the eight.  Every map against a separate kde_eval call; a few
    against the oracle at sampled pixels."""
    import torch
    t = kt.lanes(8000, 500, 2)
    b = synth.BOX_C2
    grids = {s: kde.Grid(b.lon0, b.lon1, b.lat0, b.lat1, s, s) for s in (256, 512, 1024)}
    units = {s: kde.to_grid_units(t.xy, g) for s, g in grids.items()}
    specs = synth.batch_specs(256, t.n)
    maps = _batch(specs, units, grids)
    kde.eval_batched(maps)
    torch.cuda.synchronize()
    worst = 0.0
    for k, (s, (pts, kernel, hx, hy, g, out)) in enumerate(zip(specs, maps)):
        ref = kde.eval(pts, kernel, hx, hy, g)
        torch.cuda.synchronize()
        e = kt.peak_error(out.cpu().numpy(), ref.cpu().numpy())
        worst = max(worst, e)
        assert e <= 2e-6, (k, s)
        if k % 64 == 0:
            y = out.cpu().numpy().astype(np.float64)
            og = oracle.Grid(*g.bounds, g.nx, g.ny)
            ij = kt.sample_pixels(y, 16, seed=k)
            r = kt.oracle_density_at(units[s.side][s.start:s.start + s.count], kernel, hx, hy, og, ij)
            assert kt.peak_error(y[ij[:, 1], ij[:, 0]], r) <= kt.FP32_GATE, (k, s)
    kt.log(f"256 maps: worst peak-normalised difference to separate calls {worst:.2e}")


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
