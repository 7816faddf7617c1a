"""Compression-quality measures on the GPU (kde_compression_metrics) against
the FP64 oracle.

Per-track DTW: every accumulated-cost entry is the same FP64 arithmetic on both
sides (no fused multiply-add, min exact), so the distances differ at most by
the square root's rounding: within one unit in the last place.  Lengths and
totals are sums in another order: a sum of k terms of one sign, each term
within 2 ulp, is within (k + 2) * 2^-52 of the exact sum relative to it, and
the oracle's totals are exactly rounded, so that bound (with k the terms of the
longest sum) is the tolerance.  RLL = 1 - Lc / Lo moves by at most twice the
relative error of the totals."""
import math

import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt

pytestmark = pytest.mark.gpu

U = 2.0 ** -52


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(kt.device())
    return t


def _starts(lengths):
    return np.concatenate([[0], np.cumsum(np.asarray(lengths, dtype=np.int64))]).astype(np.int64)


def _gpu(xo, lo, xc, lc):
    import torch
    r = kde.compression_metrics(_dev(np.asarray(xo, np.float64).reshape(-1, 2)), _dev(_starts(lo)),
                                _dev(np.asarray(xc, np.float64).reshape(-1, 2)), _dev(_starts(lc)))
    torch.cuda.synchronize()
    for k in ("len_o", "len_c", "dtw"):
        r[k] = r[k].cpu().numpy()
    return r


def _compare(g, r, lo, lc):
    m = len(lo)
    assert (g["n_original"], g["n_compressed"]) == (r["n_original"], r["n_compressed"])
    fin = np.isfinite(r["dtw"])
    np.testing.assert_array_equal(np.isfinite(g["dtw"]), fin)
    assert np.all(np.abs(g["dtw"][fin] - r["dtw"][fin]) <= np.spacing(r["dtw"][fin]))
    kmax = int(max(np.max(lo, initial=0), np.max(lc, initial=0)))
    for key, n in (("len_o", lo), ("len_c", lc)):
        tol = (np.asarray(n) + 2) * U * r[key]
        assert np.all(np.abs(g[key] - r[key]) <= tol), key
    ktot = kmax + m + 2
    for key in ("length_original", "length_compressed"):
        assert abs(g[key] - r[key]) <= ktot * U * r[key], key
    if m and np.all(fin):
        assert g["cr_percent"] == pytest.approx(r["cr_percent"], rel=4 * U, abs=1e-12)
        assert abs(g["rll"] - r["rll"]) <= 2 * ktot * U + 1e-300
        assert abs(g["dtw_mean"] - r["dtw_mean"]) <= (m + 2) * U * r["dtw_mean"]
        assert abs(g["dtw_std"] - r["dtw_std"]) <= 4 * (m + 2) * U * (r["dtw_mean"] + r["dtw_std"])


def _check(xo, lo, xc, lc):
    g = _gpu(xo, lo, xc, lc)
    r = oracle.track_metrics(xo, lo, xc, lc)
    _compare(g, r, lo, lc)
    return g, r


def test_hand_worked_example():
    xo = np.array([[0, 0], [1, 1], [2, 0], [4, 0], [0, 0], [0, 3]], float)
    xc = np.array([[0, 0], [4, 0], [0, 0]], float)
    g, _ = _check(xo, [4, 2], xc, [2, 1])
    assert g["dtw"][0] == math.sqrt(6.0) and g["dtw"][1] == 3.0
    assert g["cr_percent"] == 50.0


def test_strip_shapes_and_orientations():
    """Owned series of 1 .. 1100 points (one to three strips of every register
    block), swept series shorter and longer, in both orientations (a
    'compressed' series longer than its original is allowed)."""
    rng = np.random.default_rng(11)
    pairs = [(1, 1), (1, 9), (9, 1), (2, 2), (63, 200), (64, 64), (65, 300), (128, 129), (129, 130), (256, 700),
             (257, 258), (300, 100), (511, 600), (512, 513), (513, 900), (1100, 1300), (1300, 1100), (2000, 37),
             (37, 2000), (700, 64), (3, 1025)]
    xo, xc, lo, lc = [], [], [], []
    for a, b in pairs:
        p = np.cumsum(rng.normal(0, 5, (a, 2)), axis=0)
        q = np.cumsum(rng.normal(0, 5, (b, 2)), axis=0) + rng.normal(0, 3, 2)
        xo.append(p)
        xc.append(q)
        lo.append(a)
        lc.append(b)
    _check(np.concatenate(xo), lo, np.concatenate(xc), lc)


def test_dp_pipeline_matches_oracle():
    """Tracks -> GPU Douglas-Peucker -> GPU metrics, against the oracle's
    Douglas-Peucker and metrics, at several eps (the Table IV workflow)."""
    t = kt.lanes(1000, 400)
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = np.column_stack([mx, my])
    x = _dev(xy)
    st = _dev(_starts(t.lengths))
    prev_cr = -1.0
    for eps in (0.0, 1.0, 10.0, 50.0):
        keep, out, lens, cst = kde.dp_compress(x, st, eps)
        g = kde.compression_metrics(x, st, out, cst)
        import torch
        torch.cuda.synchronize()
        for k in ("len_o", "len_c", "dtw"):
            g[k] = g[k].cpu().numpy()
        ref_keep = oracle.dp_keep(xy, t.lengths, eps).astype(bool)
        lc = np.add.reduceat(ref_keep.astype(np.int64), _starts(t.lengths)[:-1])
        r = oracle.track_metrics(xy, t.lengths, xy[ref_keep], lc)
        _compare(g, r, t.lengths, lc)
        assert g["cr_percent"] >= prev_cr
        prev_cr = g["cr_percent"]
        kt.log(f"eps={eps}: CR {g['cr_percent']:.2f} %, RLL {g['rll']:.3e}, DTW {g['dtw_mean']:.3f} +- {g['dtw_std']:.3f}")


def test_empty_and_single_point_tracks():
    xo = np.array([[0, 0], [0, 1], [5, 5], [1, 1], [2, 2], [3, 3.5]], float)
    xc = np.array([[0, 0], [5, 5], [7, 7], [1, 1], [3, 3.5]], float)
    # tracks: (2 | 1), (0 | 0), (1 | 2), (0 | 0), (3 | 2)
    g, r = _check(xo, [2, 0, 1, 0, 3], xc, [1, 0, 2, 0, 2])
    assert g["dtw"][1] == 0.0 and g["dtw"][3] == 0.0
    # an empty series against a non-empty one: +inf, and mu follows
    g = _gpu(xo[:2], [2, 0], xc[:1], [0, 1])
    assert list(g["dtw"]) == [math.inf, math.inf] and g["dtw_mean"] == math.inf
    # no tracks at all
    import torch
    e = torch.zeros((0, 2), dtype=torch.float64, device=kt.device())
    z = _dev(np.zeros(1, np.int64))
    r0 = kde.compression_metrics(e, z, e, z)
    assert r0["n_original"] == 0 and math.isnan(r0["dtw_mean"]) and math.isnan(r0["cr_percent"])


def test_bench_pool_and_repeatability():
    """The bench's 4,000,000-point pool (8,000 tracks x 500) against its GPU
    Douglas-Peucker output at eps = 50 m: every per-track value and the totals
    against the oracle, and a second call bitwise equal."""
    t = kt.lanes(8000, 500, 2)
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = np.column_stack([mx, my])
    x = _dev(xy)
    st = _dev(_starts(t.lengths))
    keep, out, lens, cst = kde.dp_compress(x, st, 50.0)
    g1 = kde.compression_metrics(x, st, out, cst)
    g2 = kde.compression_metrics(x, st, out, cst)
    import torch
    torch.cuda.synchronize()
    for k in ("len_o", "len_c", "dtw"):
        assert torch.equal(g1[k], g2[k])
        g1[k] = g1[k].cpu().numpy()
    for k in ("length_original", "length_compressed", "rll", "dtw_mean", "dtw_std"):
        assert g1[k] == g2[k]
    lc = lens.cpu().numpy()
    r = oracle.track_metrics(xy, t.lengths, out.cpu().numpy(), lc)
    _compare(g1, r, t.lengths, lc)
    kt.log(f"pool: CR {g1['cr_percent']:.2f} %, RLL {g1['rll']:.3e}, DTW {g1['dtw_mean']:.3f} +- {g1['dtw_std']:.3f}")


def test_invalid_offsets_rejected():
    import torch
    x = torch.zeros((10, 2), dtype=torch.float64, device=kt.device())
    good = _dev(np.array([0, 5, 10], np.int64))
    for bad in ([0, 6, 4, 10], [1, 5, 10], [0, 5, 9]):
        st = _dev(np.array(bad, np.int64))
        with pytest.raises(kde.KDEError):
            kde.compression_metrics(x, st, x, _dev(np.array([0] * (len(bad) - 1) + [10], np.int64)))
        with pytest.raises(kde.KDEError):
            kde.compression_metrics(x, _dev(np.array([0] * (len(bad) - 1) + [10], np.int64)), x, st)
    with pytest.raises(ValueError):
        kde.compression_metrics(x, good, x, _dev(np.array([0, 10], np.int64)))


def test_totals_without_per_track_outputs():
    """per_track=False (the per-track arrays live in library workspace) gives
    the same totals bit for bit."""
    import torch
    rng = np.random.default_rng(31)
    lo = [int(v) for v in rng.integers(1, 300, 50)]
    lc = [int(v) for v in rng.integers(1, 300, 50)]
    xo = np.cumsum(rng.normal(0, 5, (sum(lo), 2)), axis=0)
    xc = np.cumsum(rng.normal(0, 5, (sum(lc), 2)), axis=0)
    args = (_dev(xo), _dev(_starts(lo)), _dev(xc), _dev(_starts(lc)))
    a = kde.compression_metrics(*args)
    b = kde.compression_metrics(*args, per_track=False)
    torch.cuda.synchronize()
    for k in ("n_original", "n_compressed", "cr_percent", "length_original", "length_compressed", "rll",
              "dtw_mean", "dtw_std"):
        assert a[k] == b[k], k
    assert "dtw" not in b
