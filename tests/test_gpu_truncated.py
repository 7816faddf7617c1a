"""The Gaussian truncated at eight bandwidths (kde_eval with KDE_TRUNCATE, FP32
direct path through support binning) against the FP64 oracle's kernel 8 and
against the full Gaussian map.  Gate: peak-normalised max error <= 1e-5."""
import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt

pytestmark = pytest.mark.gpu


def _gpu(XY, hx, hy, g, truncate=True):
    import torch
    y = kde.eval(kt.to_device(XY), 6, hx, hy, g, truncate=truncate)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


@pytest.fixture
def restore_autotune():
    yield
    kde.autotune(force=0, enabled=True)


@pytest.mark.parametrize("rc", [0, 2, 4, 8])
@pytest.mark.parametrize("H", [0.7, 2.5, 6.0])
def test_truncated_matches_oracle(rc, H, restore_autotune):
    """Ragged 300 x 170 grid, 20,000 points inside and around it; every tile shape
    (0: autotuned): support 8H from 5.6 to 48 px, binned or scanned."""
    if rc:
        kde.autotune(force=rc)
    rng = np.random.default_rng(int(10 * H) + rc)
    XY = np.column_stack([rng.uniform(-60, 360, 20000), rng.uniform(-60, 230, 20000)]).astype(np.float32)
    g, og = kde.Grid(0.0, 299.0, 0.0, 169.0, 300, 170), oracle.Grid(0.0, 299.0, 0.0, 169.0, 300, 170)
    y = _gpu(XY, H, 0.8 * H, g)
    r = kt.oracle_density_window(XY, oracle.GAUSS_TRUNC, H, 0.8 * H, og, (0, 300, 0, 170))
    e = kt.peak_error(y, r)
    kt.log(f"rc={rc} H={H}: e_inf={e:.2e}")
    assert e <= kt.FP32_GATE


def test_truncated_close_to_full_map_and_sampled_oracle():
    """10^6 lane points on 1024^2 (h = 0.002 deg, H = 2.05 px): the truncated map
    is within FP32 rounding of the full FP32 map (the dropped tails are below
    n e^-32 of the peak pair value), and matches the oracle at sampled pixels."""
    t = kt.lanes(2000, 500)
    g, og = kt.grids(synth.BOX_C2, 1024, 1024)
    XY = kde.to_grid_units(t.xy, g)
    yt = _gpu(XY, 0.002, 0.002, g)
    yf = _gpu(XY, 0.002, 0.002, g, truncate=False)
    assert kt.peak_error(yt, yf) <= 1e-6
    ij = kt.sample_pixels(yt, 48, seed=3)
    r = kt.oracle_density_at(XY, oracle.GAUSS_TRUNC, 0.002, 0.002, og, ij)
    assert kt.peak_error(yt[ij[:, 1], ij[:, 0]], r) <= kt.FP32_GATE


def test_truncated_boundary_inclusive():
    """A point on a node: nodes exactly 8 Hx away keep the factor phi(8), one
    further is 0."""
    g = kde.Grid(0.0, 40.0, 0.0, 10.0, 41, 11)
    XY = np.array([[20.0, 5.0]], dtype=np.float32)
    import torch
    y = kde.eval(kt.to_device(XY), 6, 0.5, 0.5, g, raw=True, truncate=True)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    c = oracle.k(oracle.GAUSSIAN, [0.0])[0]
    assert y[5, 24] == pytest.approx(oracle.k(oracle.GAUSSIAN, [8.0])[0] * c, rel=1e-5)
    assert y[5, 25] == 0.0 and y[5, 15] == 0.0 and y[5, 16] > 0.0


GATE_E2 = {"bf16": 2e-2, "fp16": 2e-3, "bf16x3": 2e-3, "fp16x3": 2e-3}


def _gpu_sep(XY, hx, hy, g, prec, truncate=True):
    import torch
    y = kde.eval(kt.to_device(XY), 6, hx, hy, g, precision=prec, truncate=truncate)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec", list(GATE_E2))
@pytest.mark.parametrize("H", [0.7, 2.5, 6.0, 40.0])
def test_banded_matrix_core_truncated_matches_oracle(prec, H):
    """Matrix-core paths with KDE_TRUNCATE on a ragged 300 x 170 grid: banded
    (points binned by 256 x 256 tile) for supports 8H <= 256, dense with the
    truncated factors beyond (H = 40: 8H = 320)."""
    rng = np.random.default_rng(int(10 * H) + len(prec))
    XY = np.column_stack([rng.uniform(-60, 360, 20000), rng.uniform(-60, 230, 20000)]).astype(np.float32)
    g, og = kde.Grid(0.0, 299.0, 0.0, 169.0, 300, 170), oracle.Grid(0.0, 299.0, 0.0, 169.0, 300, 170)
    y = _gpu_sep(XY, H, 0.8 * H, g, prec)
    r = kt.oracle_density_window(XY, oracle.GAUSS_TRUNC, H, 0.8 * H, og, (0, 300, 0, 170), separable=True)
    e = oracle.errors(y, r)
    kt.log(f"{prec} H={H}: e_2={e['e_2']:.2e} e_inf={e['e_inf']:.2e}")
    assert e["e_2"] <= GATE_E2[prec]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp16", "bf16x3"])
def test_banded_full_size_against_oracle(prec):
    """4*10^6 lane points on 2048^2 at h = 0.002 deg (support 32.8 px): the banded
    truncated map against the oracle's truncated Gaussian (kernel 8) on the
    256 x 256 crop holding the most points and at sampled pixels (plain loops),
    each at the precision's own e_2 gate; the dense map of the same precision
    against the full Gaussian on the same crop at that gate (the two references
    differ by less than n e^-32 of the peak pair value, far below it); repeat
    calls are bit-identical."""
    t = kt.lanes(8000, 500)
    g, og = kt.grids(synth.BOX_C2, 2048, 2048)
    XY = kde.to_grid_units(t.xy, g)
    yb = _gpu_sep(XY, 0.002, 0.002, g, prec)
    yb2 = _gpu_sep(XY, 0.002, 0.002, g, prec)
    np.testing.assert_array_equal(yb, yb2)
    yd = _gpu_sep(XY, 0.002, 0.002, g, prec, truncate=False)
    win = kt.mass_window(XY, 2048, 2048)
    crop = (slice(win[2], win[3]), slice(win[0], win[1]))
    for kernel, y in ((oracle.GAUSS_TRUNC, yb), (oracle.GAUSSIAN, yd)):
        r = kt.cached(("c3", kernel, win),
                      lambda: kt.oracle_density_window(XY, kernel, 0.002, 0.002, og, win, separable=True))
        e = oracle.errors(y[crop], r)
        kt.log(f"{prec} kernel={kernel} crop {win}: e_2={e['e_2']:.2e} e_inf={e['e_inf']:.2e}")
        assert e["e_2"] <= GATE_E2[prec]
    ij = kt.sample_pixels(yb, 32, seed=11)
    r = kt.oracle_density_at(XY, oracle.GAUSS_TRUNC, 0.002, 0.002, og, ij)
    e = oracle.errors(yb[ij[:, 1], ij[:, 0]], r)
    kt.log(f"{prec}: {ij.shape[0]} sampled pixels e_2={e['e_2']:.2e}")
    assert e["e_2"] <= GATE_E2[prec]
