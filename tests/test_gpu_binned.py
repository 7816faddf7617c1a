"""The paper's binned visualisation on the GPU (kde_bin_counts, kde_conv_counts,
kde_eval_binned) against the FP64 oracle: count matrices bit-exact (integer
work), convolutions within the FP32 gate (peak-normalised max error <= 1e-5)."""
import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt
from tests.test_oracle_pins import _golden_binned

pytestmark = pytest.mark.gpu


def _labels(tracks):
    return np.repeat(np.arange(len(tracks.lengths), dtype=np.int32), tracks.lengths)


def _dev_labels(lab):
    import torch
    return torch.from_numpy(np.ascontiguousarray(lab, dtype=np.int32)).to(kt.device())


def _gpu_counts(XY, lab, g):
    import torch
    counts, total = kde.bin_counts(kt.to_device(XY), _dev_labels(lab) if lab is not None else None, g)
    torch.cuda.synchronize()
    return counts.cpu().numpy().view(np.uint32), int(total.cpu().item())


def test_hand_worked_count_matrix():
    XY, labels, want, total = _golden_binned()
    g = kde.Grid(0.0, 7.0, 0.0, 5.0, 8, 6)
    c, t = _gpu_counts(XY, labels, g)
    np.testing.assert_array_equal(c, want)
    assert t == total
    c0, t0 = _gpu_counts(XY, None, g)
    assert t0 == 9 and int(c0.sum()) == 9


@pytest.mark.parametrize("eps", [None, 50.0])
@pytest.mark.parametrize("side", [200, 1024])
def test_counts_match_oracle_on_lanes(eps, side):
    """Lane tracks (raw, or Douglas-Peucker at 50 m so that gaps span several
    cells) with per-track labels; with and without gap filling."""
    t = kt.lanes(2000, 500) if eps is None else kt.lanes_dp(2000, 500, eps)
    g, _ = kt.grids(synth.BOX_C2, side, side)
    XY = kde.to_grid_units(t.xy, g)
    lab = _labels(t)
    for use in (lab, None):
        c, tot = _gpu_counts(XY, use, g)
        rc, rt = oracle.bin_counts(XY, use, side, side)
        kt.log(f"side={side} eps={eps} labels={use is not None}: counted {tot} cells for {XY.shape[0]} points")
        np.testing.assert_array_equal(c, rc)
        assert tot == rt


def test_counts_edge_cases():
    import torch
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 5, 4)
    c, t = _gpu_counts(np.zeros((0, 2), np.float32), None, g)
    assert t == 0 and not c.any()
    XY = np.array([[-0.999, 0.0], [0.0, -0.5], [4.0, 0.0], [np.nextafter(np.float32(4), np.float32(5)), 0.0],
                   [-1.0, 0.0], [np.nan, 1.0], [1.0, 3.0], [1e30, 2.0], [2.0, -1e30]], dtype=np.float32)
    c, t = _gpu_counts(XY, np.zeros(9, np.int32), g)
    rc, rt = oracle.bin_counts(XY, np.zeros(9, np.int32), 5, 4)
    np.testing.assert_array_equal(c, rc)
    assert t == rt
    # a long gap across the whole grid, both directions
    XY = np.array([[0.0, 0.0], [4.0, 3.0], [0.0, 3.0], [4.0, 0.0]], dtype=np.float32)
    c, t = _gpu_counts(XY, np.array([0, 0, 1, 1], np.int32), g)
    rc, rt = oracle.bin_counts(XY, np.array([0, 0, 1, 1], np.int32), 5, 4)
    np.testing.assert_array_equal(c, rc)
    assert t == rt == 10
    del torch


@pytest.mark.parametrize("kernel", range(8))
@pytest.mark.parametrize("a,b,H", [(0, 0, 1.0), (3, 3, 3.0), (7, 4, 2.5), (12, 12, 1.0), (40, 25, 30.0)])
def test_conv_matches_oracle(kernel, a, b, H):
    """Random counts on a ragged 300 x 170 grid (several tiles of both passes);
    taps up to a = 40; raw sums and the density scale."""
    import torch
    rng = np.random.default_rng(kernel * 100 + a)
    counts = rng.poisson(0.7, (170, 300)).astype(np.uint32)
    counts[rng.random((170, 300)) < 0.6] = 0
    g = kde.Grid(0.0, 299.0, 0.0, 169.0, 300, 170)
    cd = torch.from_numpy(counts.view(np.int32)).to(kt.device())
    total = torch.tensor([int(counts.sum())], dtype=torch.int64, device=kt.device())
    hx, hy = H, 0.8 * H
    raw = kde.conv_counts(cd, None, kernel, hx, hy, a, b, g, raw=True)
    dens = kde.conv_counts(cd, total, kernel, hx, hy, a, b, g)
    torch.cuda.synchronize()
    r = oracle.conv_counts(counts, kernel, np.float32(hx), np.float32(hy), a, b)  # taps carry the constants
    assert kt.peak_error(raw.cpu().numpy(), r) <= kt.FP32_GATE
    want = r / (int(counts.sum()) * hx * hy)
    assert kt.peak_error(dens.cpu().numpy(), want) <= kt.FP32_GATE


def test_eval_binned_end_to_end_and_zero_total():
    """kde_eval_binned on lane tracks (gap filling on) against the oracle's count
    matrix and convolution; an input with no point in the grid gives a zero map."""
    import torch
    t = kt.lanes_dp(500, 500, 50.0)
    g, og = kt.grids(synth.BOX_C2, 512, 512)
    XY = kde.to_grid_units(t.xy, g)
    lab = _labels(t)
    for kernel, varpi in ((6, 15), (2, 9), (7, 21)):
        hx, hy, a, b = kde.paper_taps(kernel, varpi, g)
        y = kde.eval_binned(kt.to_device(XY), _dev_labels(lab), kernel, hx, hy, a, b, g)
        torch.cuda.synchronize()
        counts, tot = oracle.bin_counts(XY, lab, 512, 512)
        Hx, Hy = oracle.bandwidth_units(hx, hy, og)
        r = oracle.conv_counts(counts, kernel, Hx, Hy, a, b, (128, 384, 128, 384)) * \
            oracle.density_scale(tot, hx, hy)
        e = kt.peak_error(y.cpu().numpy()[128:384, 128:384], r)
        kt.log(f"kernel={kernel} varpi={varpi}: e_inf={e:.2e}")
        assert e <= kt.FP32_GATE
    far = np.full((100, 2), 5000.0, dtype=np.float32)
    y = kde.eval_binned(kt.to_device(far), None, 6, g.dx, g.dy, 3, 3, g)
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0


def test_binned_equals_direct_for_points_on_nodes():
    """Points on grid nodes are not moved by the ceil projection, so with a wide
    Gaussian table the binned map equals the direct kde_eval map up to the tap
    truncation (exp(-18) of the peak at 6 sigma) and FP32 rounding."""
    import torch
    rng = np.random.default_rng(5)
    XY = rng.integers(0, 256, (20000, 2)).astype(np.float32)
    g = kde.Grid(0.0, 255.0, 0.0, 255.0, 256, 256)
    yb = kde.eval_binned(kt.to_device(XY), None, 6, 2.0, 2.0, 12, 12, g)
    yd = kde.eval(kt.to_device(XY), 6, 2.0, 2.0, g)
    torch.cuda.synchronize()
    assert kt.peak_error(yb.cpu().numpy(), yd.cpu().numpy()) <= 2e-6
