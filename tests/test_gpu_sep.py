"""Parity of the matrix-core separable path (kde_eval with the *_SEP
precisions) with the FP64 oracle.  Gates (relative L2 over the compared
outputs): plain BF16 <= 2e-2; FP16 and the hi/lo splits <= 2e-3; at full size
the FP32 direct kernel is checked beside them at e_inf <= 1e-5.  Every
result's e_2 and e_inf are printed."""
import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt

pytestmark = pytest.mark.gpu

GATE_E2 = {"bf16": 2e-2, "fp16": 2e-3, "bf16x3": 2e-3, "fp16x3": 2e-3}
PRECS = list(GATE_E2)


@pytest.mark.parametrize("prec", PRECS)
def test_small_workload_gaussian(prec):
    t = synth.workload_small()
    g, og = kt.grids(synth.BOX_C1, 128, 128)
    XY = kde.to_grid_units(t.xy, g)
    y = kt.gpu_map(XY, 6, 0.005, 0.005, g, precision=prec)
    r = kt.oracle_density_window(XY, 6, 0.005, 0.005, og, (0, 128, 0, 128))
    e = oracle.errors(y, r)
    kt.log(f"{prec}: e_2={e['e_2']:.3e} e_inf={e['e_inf']:.3e}")
    assert e["e_2"] <= GATE_E2[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kernel", list(range(8)))
def test_all_kernels_ragged(prec, kernel):
    """20,000 points on a 300 x 530 grid: two column tiles, three row tiles, all
    ragged; h about 2.4 px."""
    t = kt.lanes(100, 200)
    g, og = kt.grids(synth.BOX_C2, 300, 530)
    XY = kde.to_grid_units(t.xy, g)
    h = 0.008
    y = kt.gpu_map(XY, kernel, h, h, g, precision=prec)
    r = kt.oracle_density_window(XY, kernel, h, h, og, (0, 300, 0, 530), separable=True)
    e = oracle.errors(y, r)
    kt.log(f"{prec} kernel={kernel}: e_2={e['e_2']:.3e} e_inf={e['e_inf']:.3e}")
    assert e["e_2"] <= GATE_E2[prec]


def _c3_points():
    """4,000,000 lane points (8,000 tracks x 500) in grid units of 2048 x 2048."""
    t = kt.lanes(8000, 500)
    g, og = kt.grids(synth.BOX_C2, 2048, 2048)
    return kde.to_grid_units(t.xy, g), g, og


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp32"] + PRECS)
def test_full_size_crops(prec):
    """4,000,000 points (8,000 tracks x 500) on 2048 x 2048, Gaussian, h = 0.002
    degrees, every precision including the FP32 direct kernel: 256 x 256 crops,
    the one holding the most points and the corner [0:256, 0:256], against the
    oracle (factored form, pinned against the plain loops), plus sampled pixels
    against the plain loops.  FP32 gate: e_inf <= 1e-5 on each crop and over the
    samples; matrix-core gates: e_2 on each crop."""
    XY, g, og = _c3_points()
    kt.log(f"{prec}: n={XY.shape[0]} grid=2048x2048")
    y = kt.gpu_map(XY, 6, 0.002, 0.002, g, precision=prec)
    for win in (kt.mass_window(XY, 2048, 2048), (0, 256, 0, 256)):
        r = kt.cached(("c3", 6, win), lambda: kt.oracle_density_window(XY, 6, 0.002, 0.002, og, win,
                                                                       separable=True))
        e = oracle.errors(y[win[2]:win[3], win[0]:win[1]], r)
        kt.log(f"  crop {win}: e_2={e['e_2']:.3e} e_inf={e['e_inf']:.3e}")
        if prec == "fp32":
            assert e["e_inf"] <= kt.FP32_GATE
        else:
            assert e["e_2"] <= GATE_E2[prec]
    ij = kt.sample_pixels(y, 40, seed=5)
    r = kt.oracle_density_at(XY, 6, 0.002, 0.002, og, ij)
    e = oracle.errors(y[ij[:, 1], ij[:, 0]], r)
    kt.log(f"  {ij.shape[0]} sampled pixels (plain loops): e_2={e['e_2']:.3e} e_inf={e['e_inf']:.3e}")
    if prec == "fp32":
        assert e["e_inf"] <= kt.FP32_GATE
    else:
        assert e["e_2"] <= GATE_E2[prec]


def test_empty_and_tiny():
    import torch
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 33, 17)
    out = torch.full((17, 33), 3.0, device=kt.device())
    kde.eval(torch.empty((0, 2), device=kt.device()), 6, 0.1, 0.1, g, out=out, precision="fp16")
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    XY = np.array([[5.0, 9.0], [20.25, 3.5], [31.0, 16.0]], dtype=np.float32)
    og = oracle.Grid(0.0, 1.0, 0.0, 1.0, 33, 17)
    for prec in PRECS:
        y = kt.gpu_map(XY, 6, 2.5 * g.dx, 1.5 * g.dy, g, precision=prec)
        r = kt.oracle_density_window(XY, 6, 2.5 * g.dx, 1.5 * g.dy, og, (0, 33, 0, 17))
        assert oracle.errors(y, r)["e_2"] <= GATE_E2[prec]


def test_split_is_more_accurate_and_deterministic():
    t = kt.lanes(100, 200)
    g, og = kt.grids(synth.BOX_C2, 256, 256)
    XY = kde.to_grid_units(t.xy, g)
    r = kt.oracle_density_window(XY, 6, 0.006, 0.006, og, (0, 256, 0, 256))
    errs = {}
    for prec in PRECS:
        a = kt.gpu_map(XY, 6, 0.006, 0.006, g, precision=prec)
        b = kt.gpu_map(XY, 6, 0.006, 0.006, g, precision=prec)
        np.testing.assert_array_equal(a, b)
        errs[prec] = oracle.errors(a, r)["e_2"]
    kt.log(str(errs))
    assert errs["bf16x3"] < errs["bf16"] / 10
    assert errs["fp16x3"] < errs["fp16"] / 10


def test_main_kernel_timer_brackets_the_contraction():
    """kde_time_next_main_kernel: the armed events bracket the contraction kernel
    alone, inside the whole call, and the request is consumed by that call."""
    import torch
    t = kt.lanes(200, 500)
    g, _ = kt.grids(synth.BOX_C2, 512, 512)
    pts = kt.to_device(kde.to_grid_units(t.xy, g))
    out = torch.empty((512, 512), device=kt.device())
    stream = torch.cuda.current_stream()
    w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kde.eval(pts, 6, 0.004, 0.004, g, out=out, precision="fp16")
    w0.record(stream)
    kde.time_next_main_kernel(k0, k1)
    kde.eval(pts, 6, 0.004, 0.004, g, out=out, precision="fp16")
    w1.record(stream)
    torch.cuda.synchronize()
    whole, main = w0.elapsed_time(w1), k0.elapsed_time(k1)
    kt.log(f"whole call {whole:.3f} ms, contraction kernel {main:.3f} ms")
    assert 0.0 < main <= whole
    # consumed: a further call leaves the events where they were
    kde.eval(pts, 6, 0.004, 0.004, g, out=out, precision="fp16")
    torch.cuda.synchronize()
    assert k0.elapsed_time(k1) == main
