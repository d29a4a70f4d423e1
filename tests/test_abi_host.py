"""Host-side checks of the C ABI (no GPU): the library loads, exports every symbol
declared in include/peps.h, rejects bad arguments before enqueueing anything, and
every operand offset of the launch plan stays inside its buffer."""
import ctypes
import os
import re

import pytest

from paper_1806_03761_amd.workloads import Lattice

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _peps():
    from paper_1806_03761_amd import peps
    if not os.path.exists(peps.LIB_PATH):
        pytest.skip("library not built (python -m paper_1806_03761_amd.build)")
    return peps


def test_exports_match_header():
    peps = _peps()
    hdr = open(os.path.join(ROOT, "include", "peps.h")).read()
    declared = set(re.findall(r"\b(peps_[a-z_]+)\s*\(", hdr))
    lib = ctypes.CDLL(peps.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(peps.exported_symbols())


@pytest.mark.parametrize("lat,batch", [
    (Lattice(4, 4, 2, 4), 256), (Lattice(8, 8, 4, 16), 4096), (Lattice(16, 16, 6, 36), 4),
    (Lattice(24, 24, 8, 64), 1), (Lattice(12, 12, 6, 36), 3), (Lattice(5, 3, 3, 2), 7),
    (Lattice(2, 2, 1, 1), 3), (Lattice(3, 7, 2, 1), 5), (Lattice(7, 2, 5, 9), 2)])
def test_plan_bounds(lat, batch):
    peps = _peps()
    for grad_mode in range(4):
        for want_e in (False, True):
            assert peps.plan_check(lat, batch, grad_mode, want_e) > 0


@pytest.mark.parametrize("lat,batch", [
    (Lattice(4, 4, 2, 4), 16), (Lattice(6, 6, 2, 3), 5), (Lattice(5, 5, 3, 4), 3), (Lattice(8, 8, 4, 16), 64),
    (Lattice(16, 16, 6, 36), 2), (Lattice(12, 12, 6, 36), 3), (Lattice(4, 4, 16, 32), 2),
    (Lattice(16, 16, 16, 32), 1), (Lattice(7, 2, 5, 9), 2), (Lattice(3, 7, 2, 1), 5)])
def test_plan_bounds_variational(lat, batch):
    """The launch sequence with variational compression (1 and 2 sweeps) stays in bounds."""
    peps = _peps()
    for sweeps in (1, 2):
        for grad_mode, want_e in ((0, False), (0, True), (3, True)):
            assert peps.plan_check(lat, batch, grad_mode, want_e, sweeps) > 0


def test_plan_variational_limits():
    """Site factorisations beyond LDS (Dc D x Dc = 512 x 64) run from a global scratch
    buffer; a bond above 128 columns is refused; sweep counts outside [0, 16] are invalid."""
    peps = _peps()
    for lat in (Lattice(24, 24, 8, 64), Lattice(16, 16, 8, 64)):
        assert peps.plan_check(lat, 2, 3, True, 1) > 0
    with pytest.raises(peps.PepsError, match="unsupported"):
        peps.plan_check(Lattice(10, 10, 4, 150), 1, 0, False, 1)
    assert peps.plan_check(Lattice(10, 10, 4, 150), 1, 0, False, 0) > 0
    for sw in (-1, 17):
        with pytest.raises(peps.PepsError):
            peps.plan_check(Lattice(4, 4, 2, 4), 1, 0, False, sw)


def test_plan_rejects_bad_lattice():
    peps = _peps()
    for lat in (Lattice(1, 4, 2, 2), Lattice(4, 4, 0, 2), Lattice(4, 4, 2, 0)):
        with pytest.raises(peps.PepsError):
            peps.plan_check(lat, 1)
    with pytest.raises(peps.PepsError):
        peps.plan_check(Lattice(4, 4, 2, 2), 0)


def _bench():
    import importlib.util
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py")
    spec = importlib.util.spec_from_file_location("bench_mod", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_roofline_picks_the_binding_roof():
    """The bench's roofline takes HBM below the ridge point (peak flops / peak bandwidth)
    and the matrix cores above it, and reports achieved / peak of that roof."""
    b = _bench()
    ms, n = 1000.0, 100
    # 5 flop/byte at float64 (ridge 9.825): HBM-bound, 3 TB/s achieved
    t = {"ms_total": ms, "launches": n, "flops": 15e12, "bytes": 3e12, "tflops": 15.0, "gbps": 3000.0}
    r = b._roofline(t, 78.6)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["frac"] - 3000.0 / 8000.0) < 1e-12 and abs(r["arithmetic_intensity"] - 5.0) < 1e-12
    assert abs(r["mfma_view"]["frac"] - 15.0 / 78.6) < 1e-12
    assert abs(r["algorithmic_bytes_per_launch"] - 3e10) < 1.0
    # 20 flop/byte: matrix-core bound
    t2 = dict(t, bytes=0.75e12, gbps=750.0)
    r2 = b._roofline(t2, 78.6)
    assert r2["bound"] == "mfma" and r2["unit"] == "TFLOP/s" and abs(r2["frac"] - 15.0 / 78.6) < 1e-12
    # no byte count (the fused steps): matrix cores
    r3 = b._roofline(dict(t, bytes=0.0, gbps=0.0), 157.3)
    assert r3["bound"] == "mfma" and r3["hbm_view"] is None


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode != 0 and "one GPU" in out.stderr


def test_plan_bounds_variational_many_shapes():
    """A seeded sample of 150 lattices (Lx 2-7, Ly 2-6, D 1-5, Dc 1-30): the launch
    sequence with variational compression stays in bounds for amplitudes alone and for
    the whole path."""
    import random
    peps = _peps()
    cases = [(lx, ly, d, dc) for lx in range(2, 8) for ly in range(2, 7) for d in (1, 2, 3, 4, 5)
             for dc in (1, 2, 3, 5, 8, 16, 30)]
    random.Random(7).shuffle(cases)
    for lx, ly, d, dc in cases[:150]:
        lat = Lattice(lx, ly, d, dc)
        for gm, we in ((0, False), (3, True)):
            assert peps.plan_check(lat, 3, gm, we, 1) > 0, (lx, ly, d, dc, gm)
