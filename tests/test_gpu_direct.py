"""Parity of the FP32 direct path (kde_eval, KDE_FP32_DIRECT) with the FP64
oracle: full maps at small sizes spanning several tiles and ragged edges,
sampled pixels at the full workload sizes, and the edge cases of the method.
Gate: peak-normalised max error <= 1e-5."""
import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt

pytestmark = pytest.mark.gpu

K = list(range(8))


def test_small_workload_gaussian_full_map():
    """20 tracks x 100 points, 128 x 128 grid over 0.2 x 0.2 degrees, Gaussian,
    hx = hy = 0.005 degrees: the whole map against the oracle."""
    t = synth.workload_small()
    b = synth.BOX_C1
    g, og = kt.grids(b, 128, 128)
    XY = kde.to_grid_units(t.xy, g)
    kt.log(f"small workload: n={XY.shape[0]} grid=128x128")
    y = kt.gpu_map(XY, 6, 0.005, 0.005, g)
    r = kt.oracle_density_window(XY, 6, 0.005, 0.005, og, (0, 128, 0, 128))
    e = oracle.errors(y, r)
    kt.log(f"  e_inf={e['e_inf']:.3e} e_2={e['e_2']:.3e}")
    assert e["e_inf"] <= kt.FP32_GATE


@pytest.mark.parametrize("kernel", K)
@pytest.mark.parametrize("h", [0.004, 0.013])
def test_all_kernels_full_map_ragged(kernel, h):
    """20,000 lane points (with anchored clusters) on a 300 x 170 grid: several
    tiles in each direction and ragged last tiles; h spans about 1-2 and 4-6 px."""
    t = kt.lanes(100, 200)
    g, og = kt.grids(synth.BOX_C2, 300, 170)
    XY = kde.to_grid_units(t.xy, g)
    kt.log(f"kernel={kernel} h={h} n={XY.shape[0]} grid=300x170")
    y = kt.gpu_map(XY, kernel, h, 0.8 * h, g)
    r = kt.oracle_density_window(XY, kernel, h, 0.8 * h, og, (0, 300, 0, 170))
    e = oracle.errors(y, r)
    kt.log(f"  e_inf={e['e_inf']:.3e} e_2={e['e_2']:.3e}")
    assert e["e_inf"] <= kt.FP32_GATE


@pytest.mark.parametrize("kernel", K)
def test_full_size_lanes_sampled(kernel):
    """1,000,000 points (2,000 tracks x 500) on 1024 x 1024, h = 0.002 degrees:
    sampled pixels (peak neighbourhood, corners, quadrant peaks, random) against
    the oracle."""
    t = kt.lanes(2000, 500)
    g, og = kt.grids(synth.BOX_C2, 1024, 1024)
    XY = kde.to_grid_units(t.xy, g)
    kt.log(f"kernel={kernel} n={XY.shape[0]} grid=1024x1024")
    y = kt.gpu_map(XY, kernel, 0.002, 0.002, g)
    ij = kt.sample_pixels(y, 48, seed=kernel)
    r = kt.oracle_density_at(XY, kernel, 0.002, 0.002, og, ij)
    err = kt.peak_error(y[ij[:, 1], ij[:, 0]], r)
    kt.log(f"  sampled {ij.shape[0]} pixels, e_inf={err:.3e}")
    assert err <= kt.FP32_GATE
    # mass: the points are inside the box, so the Riemann sum of the density is ~1
    mass = y.sum() * g.dx * g.dy
    assert abs(mass - 1.0) < 2e-2


@pytest.mark.parametrize("kernel,h", [(0, 0.001), (7, 0.001), (0, 0.004), (7, 0.004), (5, 0.003)])
def test_binned_maps_with_thousands_of_tiles(kernel, h):
    """1,000,000 points on 2048 x 2048 with 32-node tiles: 4096 tiles, more than
    one workgroup's pass of the item scan, on the fixed-point path (H = 2 px;
    the cosine also at H = 8, tricube at H = 6, both at their footprint limits)
    and the gather (the uniform at H = 8): sampled pixels against the oracle,
    repeat calls bit-identical."""
    t = kt.lanes(2000, 500)
    g, og = kt.grids(synth.BOX_C2, 2048, 2048)
    XY = kde.to_grid_units(t.xy, g)
    kde.autotune(force=2)
    try:
        y = kt.gpu_map(XY, kernel, h, h, g)
        y2 = kt.gpu_map(XY, kernel, h, h, g)
    finally:
        kde.autotune(force=0)
    np.testing.assert_array_equal(y, y2)
    ij = kt.sample_pixels(y, 48, seed=kernel)
    r = kt.oracle_density_at(XY, kernel, h, h, og, ij)
    err = kt.peak_error(y[ij[:, 1], ij[:, 0]], r)
    kt.log(f"kernel={kernel} h={h}: sampled {ij.shape[0]} pixels, e_inf={err:.3e}")
    assert err <= kt.FP32_GATE


@pytest.mark.parametrize("eps", [10.0, 100.0])
def test_dp_compressed_inputs(eps):
    """Douglas-Peucker-compressed tracks (eps in metres) as input."""
    t = kt.lanes_dp(200, 500, eps)
    g, og = kt.grids(synth.BOX_C2, 256, 256)
    XY = kde.to_grid_units(t.xy, g)
    kt.log(f"dp eps={eps} n={XY.shape[0]}")
    for kernel in (6, 2):
        y = kt.gpu_map(XY, kernel, 0.006, 0.006, g)
        r = kt.oracle_density_window(XY, kernel, 0.006, 0.006, og, (0, 256, 0, 256))
        assert oracle.errors(y, r)["e_inf"] <= kt.FP32_GATE


def test_empty_input_is_zero_map():
    import torch
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 37, 21)
    out = torch.full((21, 37), 7.0, device=kt.device())
    kde.eval(torch.empty((0, 2), device=kt.device()), 6, 0.1, 0.1, g, out=out)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0


@pytest.mark.parametrize("kernel", K)
def test_single_point_on_node(kernel):
    """n = 1 at node (5, 9): peak k(0)^2/(hx hy) there, separable profile."""
    g, og = kde.Grid(0.0, 2.0, 0.0, 1.5, 41, 31), oracle.Grid(0.0, 2.0, 0.0, 1.5, 41, 31)
    XY = np.array([[5.0, 9.0]], dtype=np.float32)
    y = kt.gpu_map(XY, kernel, 0.17, 0.11, g)
    r = kt.oracle_density_window(XY, kernel, 0.17, 0.11, og, (0, 41, 0, 31))
    assert kt.peak_error(y, r) <= kt.FP32_GATE
    c = oracle.k(kernel, [0.0])[0]
    assert y[9, 5] == pytest.approx(c * c / (0.17 * 0.11), rel=2e-6)


@pytest.mark.parametrize("shape", [(2, 2), (3, 5), (129, 2), (65, 191), (1000, 7)])
@pytest.mark.parametrize("kernel", [6, 0, 5])
def test_degenerate_and_ragged_grids(shape, kernel):
    nx, ny = shape
    rng = np.random.default_rng(nx * 1000 + ny)
    XY = np.column_stack([rng.uniform(-3, nx + 2, 700), rng.uniform(-3, ny + 2, 700)]).astype(np.float32)
    g, og = kde.Grid(0.0, 1.0, 0.0, 1.0, nx, ny), oracle.Grid(0.0, 1.0, 0.0, 1.0, nx, ny)
    hx, hy = 2.3 * g.dx, 1.7 * g.dy
    y = kt.gpu_map(XY, kernel, hx, hy, g)
    r = kt.oracle_density_window(XY, kernel, hx, hy, og, (0, nx, 0, ny))
    assert y.shape == (ny, nx)
    assert kt.peak_error(y, r) <= kt.FP32_GATE


@pytest.mark.parametrize("H", [0.3, 40.0])
@pytest.mark.parametrize("kernel", [6, 2, 7])
def test_extreme_bandwidths(H, kernel):
    """Bandwidths well below one pixel and spanning a large part of the grid."""
    rng = np.random.default_rng(int(H * 10) + kernel)
    XY = rng.uniform(0, 150, (3000, 2)).astype(np.float32)
    g, og = kde.Grid(0.0, 149.0, 0.0, 149.0, 150, 150), oracle.Grid(0.0, 149.0, 0.0, 149.0, 150, 150)
    y = kt.gpu_map(XY, kernel, H, H, g)
    r = kt.oracle_density_window(XY, kernel, H, H, og, (0, 150, 0, 150))
    assert kt.peak_error(y, r) <= kt.FP32_GATE


def test_support_boundary_is_inclusive():
    """Points exactly Hx away from nodes contribute the boundary value (uniform:
    1/2 per factor), on both sides and both axes."""
    g = kde.Grid(0.0, 20.0, 0.0, 20.0, 21, 21)
    XY = np.array([[10.0, 10.0]], dtype=np.float32)
    y = kt.gpu_map(XY, 0, 2.0, 2.0, g, raw=True)
    assert y[10, 8] == 0.25 and y[10, 12] == 0.25 and y[8, 12] == 0.25
    assert y[10, 7] == 0.0 and y[13, 10] == 0.0
    assert np.count_nonzero(y) == 25


def test_raw_sum_and_determinism():
    t = kt.lanes(100, 200)
    g, _ = kt.grids(synth.BOX_C2, 256, 256)
    XY = kde.to_grid_units(t.xy, g)
    for kernel in (6, 3):
        a = kt.gpu_map(XY, kernel, 0.005, 0.005, g)
        b = kt.gpu_map(XY, kernel, 0.005, 0.005, g)
        np.testing.assert_array_equal(a, b)
        raw = kt.gpu_map(XY, kernel, 0.005, 0.005, g, raw=True)
        np.testing.assert_allclose(raw / (XY.shape[0] * 0.005 * 0.005), a, rtol=3e-7, atol=1e-30)


@pytest.mark.parametrize("kernel", [0, 1, 5, 7])
@pytest.mark.parametrize("H", [1.3, 3.5, 10.0, 60.0, 70.0])
def test_binned_and_scanned_compact_paths(kernel, H):
    """Compact kernels with n >= 4096 go through support binning when H is at
    most the tile side (H = 1.3 to 60 here) and through per-tile culling scans
    otherwise (the tile
    side follows the tuned shape); points also lie outside the grid on every
    side."""
    rng = np.random.default_rng(int(H) + 10 * kernel)
    XY = np.column_stack([rng.uniform(-90, 290, 50000), rng.uniform(-90, 240, 50000)]).astype(np.float32)
    g, og = kde.Grid(0.0, 199.0, 0.0, 149.0, 200, 150), oracle.Grid(0.0, 199.0, 0.0, 149.0, 200, 150)
    y = kt.gpu_map(XY, kernel, H, 0.9 * H, g)
    r = kt.oracle_density_window(XY, kernel, H, 0.9 * H, og, (0, 200, 0, 150))
    assert kt.peak_error(y, r) <= kt.FP32_GATE
    y2 = kt.gpu_map(XY, kernel, H, 0.9 * H, g)
    np.testing.assert_array_equal(y, y2)


@pytest.fixture
def restore_autotune():
    yield
    kde.autotune(force=0, enabled=True)


@pytest.mark.parametrize("rc", [2, 4, 8])
@pytest.mark.parametrize("kernel", [0, 2, 5, 6, 7])
@pytest.mark.parametrize("H", [1.3, 40.0])
def test_every_tile_shape_matches_oracle(rc, kernel, H, restore_autotune):
    """Each register-block shape forced (tiles of 32, 64 and 128 nodes) on a
    ragged 200 x 150 grid: compact kernels binned (H <= tile side) or scanned
    (H = 40 with 32-node tiles), the Gaussian dense."""
    kde.autotune(force=rc)
    rng = np.random.default_rng(100 * rc + 10 * kernel + int(H))
    XY = np.column_stack([rng.uniform(-50, 250, 20000), rng.uniform(-50, 200, 20000)]).astype(np.float32)
    g, og = kde.Grid(0.0, 199.0, 0.0, 149.0, 200, 150), oracle.Grid(0.0, 199.0, 0.0, 149.0, 200, 150)
    kt.log(f"rc={rc} kernel={kernel} H={H}")
    y = kt.gpu_map(XY, kernel, H, 0.8 * H, g)
    r = kt.oracle_density_window(XY, kernel, H, 0.8 * H, og, (0, 200, 0, 150))
    assert kt.peak_error(y, r) <= kt.FP32_GATE


def test_autotune_times_candidates_once_and_reuses_the_choice(restore_autotune):
    """A new bucket is tuned on the caller's data (all three shapes timed unless
    the default run is long), the fastest is cached, later calls in the bucket
    reuse it bit for bit; with tuning off no entry is added."""
    kde.autotune(clear=True, enabled=True, force=0)
    t = kt.lanes(400, 500)
    g, og = kt.grids(synth.BOX_C2, 1024, 1024)
    XY = kde.to_grid_units(t.xy, g)
    y = kt.gpu_map(XY, 2, 0.002, 0.002, g)
    ent = kde.autotune()
    keys = [k for k in ent if k.startswith("eval/") and "/compact/" in k]
    assert len(keys) == 1, ent
    e = ent[keys[0]]
    kt.log(f"{keys[0]}: {e}")
    assert e["choice"] in e["ms"] and set(e["ms"]) <= {"2", "4", "8"}
    assert e["ms"][e["choice"]] == min(e["ms"].values())
    y2 = kt.gpu_map(XY, 2, 0.002, 0.002, g)
    np.testing.assert_array_equal(y, y2)
    assert kde.autotune() == ent
    ij = kt.sample_pixels(y, 32, seed=5)
    r = kt.oracle_density_at(XY, 2, 0.002, 0.002, og, ij)
    assert kt.peak_error(y[ij[:, 1], ij[:, 0]], r) <= kt.FP32_GATE
    kde.autotune(enabled=False)
    kt.gpu_map(XY[:5000], 7, 0.02, 0.02, g)
    assert kde.autotune() == ent
