"""kde_eval_noalloc, the allocation-free kde_eval (its workspace is the
library's fixed per-GPU scratch array), against kde_eval through the C ABI:
two calls in a row, the second with a smaller input, on the FP32 direct path
(dense, support-binned and truncated), the dense matrix-core paths and the
banded matrix-core path; gates as for kde_eval (FP32: e_inf <= 1e-5; FP16 and
hi/lo: e_2 <= 2e-3).  Also: no device memory is taken by the call, maps that
need more scratch than the array holds are refused before any launch."""
import numpy as np
import pytest

import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt

pytestmark = pytest.mark.gpu

GATE = {"fp32": ("e_inf", 1e-5), "fp16": ("e_2", 2e-3), "bf16x3": ("e_2", 2e-3)}


def _errors(y, r):
    y, r = y.astype(np.float64), r.astype(np.float64)
    peak, nr = np.abs(r).max(), np.linalg.norm(r)
    return {"e_inf": float(np.abs(y - r).max() / peak) if peak > 0 else float(np.abs(y).max()),
            "e_2": float(np.linalg.norm(y - r) / nr) if nr > 0 else float(np.linalg.norm(y))}


def _case(n_tracks, pts, nx, ny):
    t = kt.lanes(n_tracks, pts)
    g, _ = kt.grids(synth.BOX_C2, nx, ny)
    return kt.to_device(kde.to_grid_units(t.xy, g)), g


@pytest.mark.parametrize("prec,kernel,truncate", [("fp32", 6, False), ("fp32", 2, False), ("fp32", 6, True),
                                                  ("fp16", 6, False), ("bf16x3", 6, False), ("fp16", 5, False)])
def test_noalloc_matches_eval_on_two_calls(prec, kernel, truncate):
    import torch
    calls = (_case(100, 200, 300, 530), _case(20, 100, 128, 96))  # 20,000 then 2,000 points
    for pts, g in calls:
        kt.log(f"{prec} kernel={kernel} truncate={truncate}: n={pts.shape[0]} grid={g.nx}x{g.ny}")
        ref = kde.eval(pts, kernel, 0.008, 0.006, g, precision=prec, truncate=truncate)
        out = torch.full((g.ny, g.nx), float("nan"), device=kt.device())
        kde.eval_noalloc(pts, kernel, 0.008, 0.006, g, out, precision=prec, truncate=truncate)
        torch.cuda.synchronize()
        y, r = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(y).all()
        e = _errors(y, r)
        name, gate = GATE[prec]
        kt.log(f"  e_inf={e['e_inf']:.2e} e_2={e['e_2']:.2e} bitwise={np.array_equal(y, r)}")
        assert e[name] <= gate


def _free_drop(entry, stream, small, big, out):
    """Free device memory lost over the second of two calls on `stream`: a small
    map first (it also sets up the stream's hardware queue and the queue's
    private-segment memory for these kernels, which the HIP runtime allocates on
    first use), then a map whose workspace is 64 MiB larger."""
    import torch
    with torch.cuda.stream(stream):
        entry(*small)
        stream.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        entry(*big, out)
        stream.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
    return free0 - free1


def test_noalloc_takes_no_device_memory_and_empty_input():
    """On streams kde_eval has never used: after a small warm-up map, a dense
    FP16 map needing 64 MiB of split planes takes no device memory through
    kde_eval_noalloc, while kde_eval (the control) grows its workspace by at
    least that much; the two maps are bitwise equal.  n = 0 writes a zero map."""
    import torch
    pts_s, g_s = _case(20, 100, 128, 96)
    pts, g = _case(100, 200, 512, 512)
    small = (pts_s, 6, 0.016, 0.016, g_s)  # about 2 px, as the large map: the same kernel variant

    def noalloc(p, k, hx, hy, grid, out=None):
        if out is None:
            out = torch.empty((grid.ny, grid.nx), device=kt.device())
        return kde.eval_noalloc(p, k, hx, hy, grid, out, precision="fp16")

    def alloc(p, k, hx, hy, grid, out=None):
        return kde.eval(p, k, hx, hy, grid, out=out, precision="fp16")

    out_n = torch.empty((512, 512), device=kt.device())
    out_a = torch.empty((512, 512), device=kt.device())
    drop_n = _free_drop(noalloc, torch.cuda.Stream(), small, (pts, 6, 0.004, 0.004, g), out_n)
    drop_a = _free_drop(alloc, torch.cuda.Stream(), small, (pts, 6, 0.004, 0.004, g), out_a)
    kt.log(f"free device memory lost over the large map: noalloc {drop_n} B, kde_eval {drop_a} B")
    assert drop_n < (2 << 20)
    assert drop_a >= (60 << 20)
    assert torch.equal(out_n, out_a)
    z = torch.full((96, 128), 5.0, device=kt.device())
    kde.eval_noalloc(torch.empty((0, 2), device=kt.device()), 6, 0.01, 0.01, g_s, z, precision="fp16")
    torch.cuda.synchronize()
    assert float(z.abs().max()) == 0.0


def test_noalloc_refuses_maps_beyond_its_scratch():
    """A dense FP16 map of 10^7 points on 512^2 needs 64 MiB of split planes and
    80 MB of padded points: refused with KDE_EINVAL before any launch (the
    output keeps its contents); the same map through kde_eval is fine."""
    import torch
    g, _ = kt.grids(synth.BOX_C2, 512, 512)
    pts = torch.full((10_000_000, 2), 256.0, device=kt.device())
    out = torch.full((512, 512), 7.0, device=kt.device())
    with pytest.raises(kde.KDEError) as ei:
        kde.eval_noalloc(pts, 6, 0.004, 0.004, g, out, precision="fp16")
    assert ei.value.status == kde.KDE_EINVAL and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert float(out.min()) == 7.0 and float(out.max()) == 7.0
