"""The C ABI on the CPU: the library loads, exports every declared symbol, and
validates arguments before touching the GPU (no compute call runs here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(kde_[a-z_]+)\s*\(", txt))
    return names


def test_exports_every_declared_symbol():
    L = kde.lib()
    names = _declared()
    assert {"kde_create_grid", "kde_eval", "kde_eval_batched", "kde_backward", "kde_lscv"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n


def _status(fn, *args):
    return getattr(kde.lib(), fn)(*args)


def test_grid_validation():
    h = ctypes.c_void_p()
    bad = [(0.0, 0.0, 0.0, 1.0, 8, 8), (0.0, 1.0, 1.0, 0.0, 8, 8), (0.0, 1.0, 0.0, 1.0, 1, 8),
           (0.0, 1.0, 0.0, 1.0, 8, 65537), (float("nan"), 1.0, 0.0, 1.0, 8, 8), (0.0, float("inf"), 0.0, 1.0, 8, 8)]
    for b in bad:
        assert _status("kde_create_grid", *b, ctypes.byref(h)) == kde.KDE_EINVAL
        assert h.value is None
        assert kde.lib().kde_last_error().decode()
    g = kde.Grid(122.0, 123.0, 30.0, 31.0, 1024, 512)
    assert (g.nx, g.ny) == (1024, 512)
    assert g.dx == (123.0 - 122.0) / 1023 and g.dy == 1.0 / 511
    assert _status("kde_grid_shape", None, None, None, None, None) == kde.KDE_EINVAL


def test_grid_units_bit_identical_to_oracle():
    t = synth.workload_lanes(n_tracks=50, pts=200)
    g = kde.Grid(122.0, 123.0, 30.0, 31.0, 1024, 1024)
    og = oracle.Grid(122.0, 123.0, 30.0, 31.0, 1024, 1024)
    np.testing.assert_array_equal(kde.to_grid_units(t.xy, g), oracle.to_units(t.xy, og))
    assert kde.bandwidth_units(0.002, 0.003, g) == oracle.bandwidth_units(0.002, 0.003, og)


def test_eval_validation_before_launch():
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 64, 64)
    L = kde.lib()
    ok = dict(points=FAKE, n=10, k=6, hx=0.05, hy=0.05, g=g.handle, out=FAKE, prec=0, flags=0, s=None)

    def call(**kw):
        a = dict(ok, **kw)
        return L.kde_eval(a["points"], a["n"], a["k"], a["hx"], a["hy"], a["g"], a["out"], a["prec"], a["flags"],
                          a["s"])

    for kw in (dict(n=-1), dict(n=1 << 31), dict(points=None), dict(k=8), dict(k=-1), dict(hx=0.0),
               dict(hy=-1.0), dict(hx=float("nan")), dict(hy=float("inf")), dict(hx=1e-9), dict(hx=1e9),
               dict(g=None), dict(out=None), dict(prec=5), dict(prec=-1), dict(flags=2)):
        assert call(**kw) == kde.KDE_EINVAL, kw
        assert L.kde_last_error().decode()


def test_other_entry_points_validate():
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 64, 64)
    L = kde.lib()
    assert L.kde_backward(FAKE, 10, 6, 0.05, 0.05, g.handle, None, FAKE, None, 0, None) == kde.KDE_EINVAL
    assert L.kde_backward(FAKE, 10, 9, 0.05, 0.05, g.handle, FAKE, FAKE, None, 0, None) == kde.KDE_EINVAL
    assert L.kde_backward(FAKE, 10, 6, 0.05, 0.05, g.handle, FAKE, FAKE, None, 32, None) == kde.KDE_EINVAL
    assert "unknown flags" in L.kde_last_error().decode()
    v = ctypes.c_double()
    assert L.kde_lscv(FAKE, 1, 6, 0.05, 0.05, g.handle, ctypes.byref(v), None, None) == kde.KDE_EINVAL
    assert L.kde_lscv(FAKE, 10, 6, 0.05, 0.05, g.handle, None, None, None) == kde.KDE_EINVAL
    assert L.kde_eval_batched(None, 3, 0, None) == kde.KDE_EINVAL
    m = (kde.MapDesc * 2)()
    for d in m:
        d.points, d.n, d.kernel_id, d.hx, d.hy, d.grid, d.out = FAKE.value, 5, 6, 0.05, 0.05, g.handle.value, FAKE.value
    m[1].kernel_id = 11
    assert L.kde_eval_batched(m, 2, 0, None) == kde.KDE_EINVAL
    assert "kernel" in L.kde_last_error().decode()
    m[1].kernel_id = 2
    for field, value, words in (("precision", 5, "precision"), ("precision", -1, "precision"),
                                ("flags", 2, "flags"), ("flags", 8, "KDE_TRUNCATE"), ("reserved", 1, "reserved")):
        setattr(m[1], field, value)
        assert L.kde_eval_batched(m, 2, 0, None) == kde.KDE_EINVAL, (field, value)
        assert words in L.kde_last_error().decode(), (field, value)
        setattr(m[1], field, 0)
    assert ctypes.sizeof(kde.MapDesc) == 64


def test_main_kernel_timer_arguments():
    L = kde.lib()
    assert L.kde_time_next_main_kernel(FAKE, None) == kde.KDE_EINVAL
    assert "both events" in L.kde_last_error().decode()
    assert L.kde_time_next_main_kernel(None, FAKE) == kde.KDE_EINVAL
    assert L.kde_time_next_main_kernel(None, None) == kde.KDE_OK


def test_autotune_cache_roundtrip_and_rejection(tmp_path):
    """The autotuner's JSON cache: entries load, dump and save; a corrupt file,
    a foreign format tag or an invalid choice is rejected whole (cache unchanged);
    bad switches are refused."""
    import json
    L = kde.lib()
    kde.autotune(clear=True)
    good = {"format": "kde-autotune-1", "entries": {
        "eval/gfx950/compact/H2/n20/px20": {"choice": "2", "ms": {"2": 1.25, "4": 2.5, "8": 3.75}},
        "batch/gfx950/00112233aabbccdd": {"choice": "8,4", "ms": {"8,4": 36.0, "8,2": 44.5}}}}
    f = tmp_path / "good.json"
    f.write_text(json.dumps(good))
    ent = kde.autotune(load=str(f))
    assert ent == good["entries"]
    out = tmp_path / "saved.json"
    kde.autotune(save=str(out))
    assert json.loads(out.read_text()) == good
    for bad in ('{"format": "kde-autotune-1", "entries": {', "not json",
                '{"format": "kde-autotune-0", "entries": {}}',
                '{"format": "kde-autotune-1", "entries": {"eval/x": {"choice": "3", "ms": {}}}}',
                '{"format": "kde-autotune-1", "entries": {"batch/x": {"choice": "8,5", "ms": {}}}}',
                '{"format": "kde-autotune-1", "entries": {"other/x": {"choice": "2", "ms": {}}}}',
                '{"format": "kde-autotune-1", "entries": {"eval/x": {"ms": {}}}}'):
        b = tmp_path / "bad.json"
        b.write_text(bad)
        assert L.kde_autotune_load(os.fsencode(str(b))) == kde.KDE_EINVAL, bad
        assert L.kde_last_error().decode()
        assert kde.autotune() == good["entries"]
    assert L.kde_autotune_load(os.fsencode(str(tmp_path / "missing.json"))) == kde.KDE_EINVAL
    assert L.kde_autotune_force(3) == kde.KDE_EINVAL and L.kde_autotune_force(16) == kde.KDE_EINVAL
    assert L.kde_autotune_enable(2) == kde.KDE_EINVAL
    need = ctypes.c_size_t()
    assert L.kde_autotune_dump(None, 0, ctypes.byref(need)) == kde.KDE_OK and need.value > 10
    small = ctypes.create_string_buffer(4)
    assert L.kde_autotune_dump(small, 4, ctypes.byref(need)) == kde.KDE_EINVAL
    assert kde.autotune(clear=True) == {}


def test_truncate_flag_validation():
    L = kde.lib()
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 16, 16)
    assert L.kde_eval(FAKE, 10, 2, 0.1, 0.1, g.handle, FAKE, 0, 8, None) == kde.KDE_EINVAL  # not Gaussian
    assert "KDE_TRUNCATE" in L.kde_last_error().decode()
    assert L.kde_eval(FAKE, 10, 6, 0.1, 0.1, g.handle, FAKE, 0, 16, None) == kde.KDE_EINVAL  # unknown flag


def test_dp_entry_point_validates():
    L = kde.lib()
    n = ctypes.c_int64()
    assert L.kde_dp_compress(FAKE, -1, FAKE, 1, 1.0, FAKE, None, None, None, None, None) == kde.KDE_EINVAL
    assert L.kde_dp_compress(FAKE, 10, FAKE, 0, 1.0, FAKE, None, None, None, None, None) == kde.KDE_EINVAL
    assert L.kde_dp_compress(FAKE, 10, FAKE, 11, 1.0, FAKE, None, None, None, None, None) == kde.KDE_EINVAL
    assert L.kde_dp_compress(FAKE, 10, FAKE, 2, -1.0, FAKE, None, None, None, None, None) == kde.KDE_EINVAL
    assert L.kde_dp_compress(FAKE, 10, FAKE, 2, float("nan"), FAKE, None, None, None, None, None) == kde.KDE_EINVAL
    assert L.kde_dp_compress(None, 10, FAKE, 2, 1.0, FAKE, None, None, None, None, None) == kde.KDE_EINVAL
    assert L.kde_dp_compress(None, 0, None, 0, 1.0, None, None, None, None, ctypes.byref(n), None) == kde.KDE_OK
    assert n.value == 0


def test_metrics_entry_point_validates():
    L = kde.lib()
    f = L.kde_compression_metrics
    assert f(FAKE, -1, FAKE, FAKE, 0, FAKE, 1, None, None, None, None, None) == kde.KDE_EINVAL
    assert f(FAKE, 10, FAKE, FAKE, -1, FAKE, 1, None, None, None, None, None) == kde.KDE_EINVAL
    assert f(FAKE, 10, FAKE, FAKE, 10, FAKE, -1, None, None, None, None, None) == kde.KDE_EINVAL
    assert f(FAKE, 10, None, FAKE, 10, FAKE, 1, None, None, None, None, None) == kde.KDE_EINVAL
    assert f(FAKE, 10, FAKE, FAKE, 10, None, 1, None, None, None, None, None) == kde.KDE_EINVAL
    assert f(None, 10, FAKE, FAKE, 10, FAKE, 1, None, None, None, None, None) == kde.KDE_EINVAL
    assert f(FAKE, 10, FAKE, None, 10, FAKE, 1, None, None, None, None, None) == kde.KDE_EINVAL
    assert "kde_compression_metrics" in L.kde_last_error().decode()


def test_binned_entry_points_validate():
    L = kde.lib()
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 16, 16)
    assert L.kde_bin_counts(FAKE, 10, None, None, FAKE, None, None) == kde.KDE_EINVAL
    assert L.kde_bin_counts(None, 10, None, g.handle, FAKE, None, None) == kde.KDE_EINVAL
    assert L.kde_bin_counts(FAKE, 10, None, g.handle, None, None, None) == kde.KDE_EINVAL
    assert L.kde_conv_counts(FAKE, FAKE, g.handle, 6, 0.1, 0.1, 129, 3, FAKE, 0, None) == kde.KDE_EINVAL
    assert "tap radii" in L.kde_last_error().decode()
    assert L.kde_conv_counts(FAKE, FAKE, g.handle, 6, 0.1, 0.1, 3, -1, FAKE, 0, None) == kde.KDE_EINVAL
    assert L.kde_conv_counts(FAKE, None, g.handle, 6, 0.1, 0.1, 3, 3, FAKE, 0, None) == kde.KDE_EINVAL
    assert L.kde_conv_counts(FAKE, FAKE, g.handle, 8, 0.1, 0.1, 3, 3, FAKE, 0, None) == kde.KDE_EINVAL
    assert L.kde_conv_counts(FAKE, FAKE, g.handle, 6, 0.1, 0.1, 3, 3, FAKE, 8, None) == kde.KDE_EINVAL
    assert L.kde_eval_binned(FAKE, 10, None, 6, 0.1, 0.1, 3, 3, g.handle, None, 0, None) == kde.KDE_EINVAL
    assert L.kde_eval_binned(FAKE, 10, None, 6, -0.1, 0.1, 3, 3, g.handle, FAKE, 0, None) == kde.KDE_EINVAL
    assert kde.paper_taps("gaussian", 7, g) == (g.dx, g.dy, 3, 3)
    assert kde.paper_taps("epanechnikov", 7, g) == (3 * g.dx, 3 * g.dy, 3, 3)
    with pytest.raises(ValueError):
        kde.paper_taps(2, 8, g)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(kde, "_lib", None)
    monkeypatch.setattr(kde, "LIB_PATH", str(tmp_path / "libkde.so"))
    with pytest.raises(RuntimeError, match="libkde.so not found"):
        kde.lib()


def test_single_hip_runtime_in_process():
    """libkde binds to the HIP runtime PyTorch already loaded (same soname), so a
    process that uses both holds one copy of libamdhip64."""
    import subprocess
    import sys
    code = ("import paper_2004_13653_amd as kde, oracle, synth\n"
            "kde.Grid(0.0, 1.0, 0.0, 1.0, 8, 8)\n"
            "import torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_noalloc_entry_point_validates_before_launch():
    """kde_eval_noalloc validates like kde_eval, and refuses a map whose
    workspace exceeds its fixed scratch array before anything is launched
    (dense FP16 at 2*10^7 points on 512^2: 64 MiB of split planes plus 160 MB
    of padded points)."""
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 512, 512)
    L = kde.lib()
    for args in ((FAKE, -1, 6, 0.05, 0.05, g.handle, FAKE, 0, 0, None),
                 (None, 10, 6, 0.05, 0.05, g.handle, FAKE, 0, 0, None),
                 (FAKE, 10, 9, 0.05, 0.05, g.handle, FAKE, 0, 0, None),
                 (FAKE, 10, 6, 0.0, 0.05, g.handle, FAKE, 0, 0, None),
                 (FAKE, 10, 6, 0.05, 0.05, None, FAKE, 0, 0, None),
                 (FAKE, 10, 6, 0.05, 0.05, g.handle, None, 0, 0, None),
                 (FAKE, 10, 6, 0.05, 0.05, g.handle, FAKE, 7, 0, None),
                 (FAKE, 10, 2, 0.05, 0.05, g.handle, FAKE, 0, 8, None)):
        assert L.kde_eval_noalloc(*args) == kde.KDE_EINVAL, args
        assert L.kde_last_error().decode().startswith("kde_eval_noalloc")
    assert L.kde_eval_noalloc(FAKE, 20_000_000, 6, 0.004, 0.004, g.handle, FAKE, 1, 0, None) == kde.KDE_EINVAL
    assert "scratch" in L.kde_last_error().decode()
    assert kde.NOALLOC_SCRATCH_BYTES == 128 << 20
