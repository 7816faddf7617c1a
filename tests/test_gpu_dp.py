"""Douglas-Peucker compression on the GPU (kde_dp_compress) against the FP64
oracle: keep masks bit-exact (the decision is integer-exact in both), the
compacted points and per-track counts exact."""
import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt

pytestmark = pytest.mark.gpu


def _run(xy, lengths, eps):
    import torch
    start = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    x = torch.from_numpy(np.ascontiguousarray(xy, dtype=np.float64)).to(kt.device())
    st = torch.from_numpy(start).to(kt.device())
    keep, out, lens, cst = kde.dp_compress(x, st, eps)
    torch.cuda.synchronize()
    lens = lens.cpu().numpy()
    # the compressed tracks' offsets are the running sums of their lengths
    np.testing.assert_array_equal(cst.cpu().numpy(), np.concatenate([[0], np.cumsum(lens)]))
    return keep.cpu().numpy(), out.cpu().numpy(), lens


def _check(xy, lengths, eps):
    keep, out, lens = _run(xy, lengths, eps)
    ref = oracle.dp_keep(xy, lengths, eps)
    np.testing.assert_array_equal(keep, ref)
    np.testing.assert_array_equal(out, np.asarray(xy, dtype=np.float64)[ref.astype(bool)])
    start = np.concatenate([[0], np.cumsum(lengths)])
    np.testing.assert_array_equal(lens, [int(ref[a:b].sum()) for a, b in zip(start, start[1:])])
    return keep


def test_textbook_cases():
    y = np.zeros(9)
    y[4] = 5.0
    cases = [(np.column_stack([np.arange(10.0), 2 * np.arange(10.0)]), 0.0),
             (np.column_stack([np.arange(9.0), y]), 4.999), (np.column_stack([np.arange(9.0), y]), 5.0),
             (np.array([[0, 0], [1, 1], [2, 0], [3, 1], [4, 0]], float), 0.7),
             (np.array([[0, 0], [10, 0], [5, 0]], float), 0.0),
             (np.array([[0, 0], [3, 4], [0, 0]], float), 4.9), (np.array([[0, 0], [3, 4], [0, 0]], float), 5.0)]
    for xy, eps in cases:
        _check(xy, [len(xy)], eps)


def test_track_shapes_and_degenerate_chords():
    """Tracks of 1, 2, 3 and many points, empty tracks, repeated points (zero
    chords) and a closed loop, merged in one buffer."""
    rng = np.random.default_rng(4)
    parts, lens = [], []
    for L in (1, 2, 0, 3, 50, 0, 7, 200):
        p = np.cumsum(rng.normal(0, 1, (L, 2)), axis=0)
        if L >= 7:
            p[3] = p[2]          # a repeated point
            p[-1] = p[0]         # closed loop: zero chord at the top level
        parts.append(p)
        lens.append(L)
    xy = np.concatenate([p for p in parts if len(p)])
    for eps in (0.0, 0.5, 3.0, 1e9):
        _check(xy, lens, eps)


def test_long_and_short_tracks():
    """Tracks of up to 1024 points run whole in one workgroup each; longer ones
    (1025, 3000 and 5000 points here) take the level-synchronous kernels.  A mix
    of both, including one exactly 1024 long, in one call."""
    rng = np.random.default_rng(11)
    lens = [5000, 12, 1024, 1025, 0, 300, 3000, 2, 1023]
    parts = []
    for L in lens:
        p = np.cumsum(rng.normal(0, 20.0, (L, 2)), axis=0)
        if L >= 300:
            p[L // 2] = p[L // 2 - 1]  # a repeated point
        parts.append(p)
    xy = np.concatenate([p for p in parts if len(p)])
    for eps in (0.0, 10.0, 50.0):
        keep = _check(xy, lens, eps)
        kt.log(f"eps={eps}: kept {int(keep.sum())} of {keep.size}")


@pytest.mark.parametrize("eps", [0.0, 10.0, 50.0, 100.0])
def test_lane_tracks_match_oracle(eps):
    """2,000 lane tracks x 500 reports in Mercator metres."""
    t = kt.lanes(2000, 500)
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    keep = _check(np.column_stack([mx, my]), t.lengths, eps)
    kt.log(f"eps={eps}: kept {int(keep.sum())} of {keep.size}")


def test_full_pool_and_repeatability():
    """The 4,000,000-point pool (8,000 tracks) at eps = 50 m, twice."""
    t = kt.lanes(8000, 500, 2)
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = np.column_stack([mx, my])
    k1 = _check(xy, t.lengths, 50.0)
    k2, _, _ = _run(xy, t.lengths, 50.0)
    np.testing.assert_array_equal(k1, k2)


def test_invalid_offsets_rejected():
    import torch
    x = torch.zeros((10, 2), dtype=torch.float64, device=kt.device())
    for bad in ([0, 6, 4, 10], [1, 5, 10], [0, 5, 9]):
        st = torch.tensor(bad, dtype=torch.int64, device=kt.device())
        with pytest.raises(kde.KDEError):
            kde.dp_compress(x, st, 1.0)


def test_empty_input_offsets():
    """No points and no tracks: nothing kept, and the compressed offsets are [0]."""
    import torch
    x = torch.zeros((0, 2), dtype=torch.float64, device=kt.device())
    st = torch.zeros(1, dtype=torch.int64, device=kt.device())
    keep, out, lens, cst = kde.dp_compress(x, st, 10.0)
    torch.cuda.synchronize()
    assert keep.numel() == 0 and out.shape[0] == 0 and lens.numel() == 0
    assert cst.cpu().tolist() == [0]
