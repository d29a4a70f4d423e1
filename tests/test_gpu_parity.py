"""GPU path (through the C ABI) against the FP64 oracle, element by element.

Tolerances (log-amplitude |d| <= tol * max(1, |ln W|), sign equal):
  f64 1e-10, f32 1e-5, bf16 2e-2.  Local energy: f64 1e-9, f32 1e-4 relative to
  max(1, |E|).  Log-derivatives: per-sample relative l2 error f64 1e-9, f32 1e-4.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_1806_03761_amd.workloads import Lattice, make_random, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_AMP = {"f64": 1e-10, "f32": 1e-5, "bf16": 2e-2}
TOL_E = {"f64": 1e-9, "f32": 1e-4, "bf16": None}
TOL_G = {"f64": 1e-9, "f32": 1e-4, "bf16": None}


def _peps():
    from paper_1806_03761_amd import peps
    return peps


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(A, S):
    return torch.from_numpy(A).cuda(), torch.from_numpy(np.ascontiguousarray(S)).cuda()


def _np(*ts):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ts]


def _assert_amp(la, sg, la_o, sg_o, tol):
    assert np.array_equal(sg.astype(int), sg_o.astype(int)), (sg, sg_o)
    err = np.abs(la - la_o) / np.maximum(1.0, np.abs(la_o))
    assert err.max() <= tol, f"max log-amp error {err.max():.3e} > {tol}"
    return err.max()


def _assert_e(e, e_o, tol):
    err = np.abs(e - e_o) / np.maximum(1.0, np.abs(e_o))
    assert err.max() <= tol, f"max E_loc error {err.max():.3e} > {tol}"
    return err.max()


# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_amplitude_4x4_workload(prec):
    lat, A, S, _ = make_workload("4x4_D2_Dc4")
    _say("4x4 D2 Dc4 amplitude", prec, S.shape)
    la, sg, fl = _np(*_peps().log_amplitude(*_dev(A, S), lat, prec))
    la_o, sg_o, fl_o = O.log_amplitude(A, lat, S)
    assert np.all(fl == 0) and np.all(fl_o == 0)
    _assert_amp(la, sg, la_o, sg_o, TOL_AMP[prec])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_local_energy_4x4_workload(prec):
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 96)
    _say("4x4 local energy", prec)
    la, sg, e, fl = _np(*_peps().local_energy(*_dev(A, S), lat, prec))
    la_o, sg_o, e_o, fl_o = O.local_energy(A, lat, S)
    assert np.all(fl == 0)
    _assert_amp(la, sg, la_o, sg_o, TOL_AMP[prec])
    _assert_e(e, e_o, TOL_E[prec])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_log_derivative_4x4_per_sample(prec):
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 12)
    _say("4x4 log-derivative", prec)
    out, la, sg, fl = _np(*_peps().log_derivative(*_dev(A, S), lat, prec))
    ref = O.log_derivative(A, lat, S)
    for b in range(len(S)):
        err = np.linalg.norm(out[b] - ref[b]) / np.linalg.norm(ref[b])
        assert err <= TOL_G[prec], (b, err)
        # entries that must be exactly zero: the other slice and dead leg entries
        assert np.all(out[b][ref[b] == 0] == 0)


def test_ragged_8x8_D4_f64():
    """Truncated regime (Dc = 16 < 4^4), batch 37: several tiles and a ragged tail."""
    lat, A, S, _ = make_workload("8x8_D4_Dc16", 37)
    _say("8x8 D4 Dc16 f64 amplitude b=37")
    la, sg, fl = _np(*_peps().log_amplitude(*_dev(A, S), lat, "f64"))
    la_o, sg_o, _ = O.log_amplitude(A, lat, S)
    assert np.all(fl == 0)
    _assert_amp(la, sg, la_o, sg_o, 1e-10)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_path_8x8_D4(prec):
    lat, A, S, _ = make_workload("8x8_D4_Dc16", 6)
    _say("8x8 full path", prec)
    la, sg, e, d, fl = _np(*_peps().evaluate(*_dev(A, S), lat, prec, grad_mode=1))
    for b in range(len(S)):
        la_o, sg_o, e_o, d_o, fl_o = O.full_path_one(A, lat, S[b])
        assert fl[b] == 0 and fl_o == 0
        assert sg[b] == sg_o
        assert abs(la[b] - la_o) <= TOL_AMP[prec] * max(1, abs(la_o))
        assert abs(e[b] - e_o) <= TOL_E[prec] * max(1, abs(e_o))
        assert np.linalg.norm(d[b] - d_o) <= TOL_G[prec] * np.linalg.norm(d_o)


def test_vjp_and_energy_gradient_4x4():
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 40)
    _say("4x4 VJP and dE/dA")
    Ad, Sd = _dev(A, S)
    w = np.random.default_rng(0).standard_normal(len(S))
    g, _, _, _ = _peps().log_derivative(Ad, Sd, lat, "f64", weights=torch.from_numpy(w).cuda())
    (g,) = _np(g)
    per = O.log_derivative(A, lat, S)
    ref = np.einsum("b,bnse->nse", w, per)
    assert np.linalg.norm(g - ref) <= 1e-10 * np.linalg.norm(ref)
    la, sg, e, gE, fl = _np(*_peps().evaluate(Ad, Sd, lat, "f64", grad_mode=3))
    _, _, e_o, _ = O.local_energy(A, lat, S)
    Bn = len(S)
    refE = 2.0 * np.einsum("b,bnse->nse", e_o, per) / Bn - 2.0 * (per.sum(0) / Bn) * e_o.mean()
    assert np.linalg.norm(gE - refE) <= 1e-9 * np.linalg.norm(refE)


def test_chunked_batch_matches_single_chunk():
    """A workspace limit that forces several chunks gives the same results."""
    p = _peps()
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 50)
    Ad, Sd = _dev(A, S)
    la1, sg1, e1, g1, _ = _np(*p.evaluate(Ad, Sd, lat, "f64", grad_mode=3))
    per = p.workspace_bytes(lat, 1)
    p.set_workspace_limit(per * 8)
    try:
        la2, sg2, e2, g2, _ = _np(*p.evaluate(Ad, Sd, lat, "f64", grad_mode=3))
    finally:
        p.set_workspace_limit(0)
    assert np.array_equal(la1, la2) and np.array_equal(e1, e2)
    assert np.allclose(g1, g2, rtol=1e-12, atol=1e-14)


def test_closed_form_neel_and_flags():
    """Neel product state (embedded at D = 3, dense gauges) at S = Neel: E = -N_J1/4 + J2 N_J2/4;
    a non-Neel S has zero amplitude (flag 2); a config value of 2 is flag 1."""
    import pins_lib as P
    lat = Lattice(6, 4, 3, 4)
    rng = np.random.default_rng(4)
    a = np.zeros((lat.N, 2))
    for m in range(lat.N):
        i, j = divmod(m, lat.Lx)
        a[m, (i + j) % 2] = 1.0
    A = P.gauge_dress(P.product_peps(lat, a, rng, 0.3), lat, rng)
    neel = np.array([(i + j) % 2 for i in range(lat.Ly) for j in range(lat.Lx)], np.int8)
    S = np.stack([neel, neel.copy(), neel.copy()])
    S[1, [0, 1]] = S[1, [1, 0]]
    S[2, 5] = 2
    la, sg, e, fl = _np(*_peps().local_energy(*_dev(A, S), lat, "f64"))
    nj1 = lat.Ly * (lat.Lx - 1) + lat.Lx * (lat.Ly - 1)
    nj2 = 2 * (lat.Lx - 1) * (lat.Ly - 1)
    assert fl.tolist() == [0, 2, 1], (fl, la, sg, e)
    assert abs(la[0]) < 1e-12 and sg[0] == 1
    assert abs(e[0] - (-nj1 / 4 + lat.J2 * nj2 / 4)) < 1e-11
    assert sg[1] == 0 and la[1] == -math.inf and math.isnan(e[1])
    assert math.isnan(la[2]) and math.isnan(e[2])


def test_empty_batch_is_noop():
    lat = Lattice(4, 4, 2, 4)
    A, S = make_random(lat, 0, 1)
    la, sg, fl = _np(*_peps().log_amplitude(*_dev(A, S.reshape(0, 16)), lat, "f64"))
    assert la.shape == (0,)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_random_product_state_closed_form(prec):
    """Random D = 1 product state embedded at D = 3 (Dc = 2, so truncation is active
    but exact), gauge-dressed: ln|W| = sum ln|a|, E(S) closed form, Euler rule."""
    import pins_lib as P
    lat = Lattice(5, 4, 3, 2)
    rng = np.random.default_rng(7)
    a = rng.uniform(0.5, 1.5, size=(lat.N, 2)) * rng.choice([-1, 1], size=(lat.N, 2))
    A = P.gauge_dress(P.product_peps(lat, a, rng, 0.3), lat, rng)
    _, S = make_random(lat, 5, 17)
    la, sg, e, d, fl = _np(*_peps().evaluate(*_dev(A, S), lat, prec, grad_mode=1))
    assert np.all(fl == 0), fl
    nn, nnn = P.lattice_bonds(lat.Lx, lat.Ly)
    for b in range(len(S)):
        s = S[b]
        vals = a[np.arange(lat.N), s]
        assert abs(la[b] - np.sum(np.log(np.abs(vals)))) <= TOL_AMP[prec] * max(1, abs(la[b]))
        sig = 1 - 2 * s.astype(int)
        E = 0.0
        for bonds, J in ((nn, lat.J1), (nnn, lat.J2)):
            for m, n in bonds:
                E += J * sig[m] * sig[n] / 4
                if s[m] != s[n]:
                    E += J * 0.5 * a[m, 1 - s[m]] * a[n, 1 - s[n]] / (a[m, s[m]] * a[n, s[n]])
        assert abs(e[b] - E) <= TOL_E[prec] * max(1, abs(E))
        for m in range(lat.N):
            t = A[m, s[m]].reshape(-1)
            # Euler rule on the live block (dead entries of A hold junk, Delta is 0 there)
            assert abs(np.dot(t, d[b, m, s[m]]) - 1.0) <= (1e-9 if prec == "f64" else 1e-4)


def test_bf16_error_report_8x8():
    """bf16 contraction GEMMs (fp32 accumulation, fp64 factorisations): log-amplitude
    within 2e-2 of the oracle (sign equal); E_loc and gradient errors are reported."""
    lat, A, S, _ = make_workload("8x8_D4_Dc16", 6)
    la, sg, e, d, fl = _np(*_peps().evaluate(*_dev(A, S), lat, "bf16", grad_mode=1))
    errs_l, errs_e, errs_g = [], [], []
    for b in range(len(S)):
        la_o, sg_o, e_o, d_o, fl_o = O.full_path_one(A, lat, S[b])
        assert fl[b] == 0 and sg[b] == sg_o
        errs_l.append(abs(la[b] - la_o) / max(1.0, abs(la_o)))
        errs_e.append(abs(e[b] - e_o) / max(1.0, abs(e_o)))
        errs_g.append(np.linalg.norm(d[b] - d_o) / np.linalg.norm(d_o))
    _say("bf16 8x8: log-amp rel err max %.2e, E_loc rel err max %.2e, grad rel l2 max %.2e"
         % (max(errs_l), max(errs_e), max(errs_g)))
    _say("bf16 8x8: E_loc rel err median %.2e; grad rel l2 median %.2e"
         % (np.median(errs_e), np.median(errs_g)))
    assert max(errs_l) <= TOL_AMP["bf16"]
    # E_loc and gradient in bf16 mode are reported, not held to a tolerance (the ratios
    # of uniformly drawn configurations are heavy-tailed); they must be finite
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(d))


def test_autograd_function_4x4():
    """PepsLogAmp.backward = the oracle's weighted log-derivative, and agrees with a
    central finite difference (h = 1e-6, f64) of the GPU forward itself (exact regime,
    where the frozen-environment derivative is the full derivative)."""
    p = _peps()
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 8)
    Ad, Sd = _dev(A, S)
    Ad.requires_grad_(True)
    la, sg, fl = p.PepsLogAmp.apply(Ad, Sd, lat, "f64")
    g = torch.from_numpy(np.random.default_rng(1).standard_normal(len(S))).cuda()
    (la * g).sum().backward()
    grad = Ad.grad.detach().cpu().numpy().reshape(lat.N, 2, -1)
    ref = np.einsum("b,bnse->nse", g.cpu().numpy(), O.log_derivative(A, lat, S))
    assert np.linalg.norm(grad - ref) <= 1e-10 * np.linalg.norm(ref)
    rng = np.random.default_rng(2)
    h = 1e-6
    gw = g.cpu().numpy()
    for _ in range(12):
        m = int(rng.integers(lat.N))
        s = int(S[int(rng.integers(len(S))), m])
        dims = O.leg_dims(lat, m // lat.Lx, m % lat.Lx)
        idx = tuple(int(rng.integers(dk)) for dk in dims)
        Ap = A.copy(); Am = A.copy()
        Ap[(m, s) + idx] += h
        Am[(m, s) + idx] -= h
        lp, _, _ = p.log_amplitude(*_dev(Ap, S), lat, "f64")
        lm, _, _ = p.log_amplitude(*_dev(Am, S), lat, "f64")
        fd = float(((lp - lm).cpu().numpy() / (2 * h)) @ gw)
        an = float(grad[m, s].reshape(lat.D, lat.D, lat.D, lat.D)[idx])
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (m, s, idx, fd, an)


# At 16x16, D = 6, Dc = 36 the truncation amplifies input rounding: rounding only the
# apply operands to f32 (all arithmetic in f64) already moves ln|W| by 1.2e-5 relative on
# the first configuration.  The float32 path is held to the stated 1e-5 bound and is
# expected to miss it (measured about 3e-5): recorded as an expected failure, not passed
# under a wider bound.
TOL_AMP_16 = {"f64": 1e-10, "f32": 1e-5}


@pytest.mark.parametrize("prec", ["f64", pytest.param("f32", marks=pytest.mark.xfail(
    reason="float32 apply rounding amplified by the Dc = 36 truncation exceeds 1e-5", strict=False))])
def test_amplitude_16x16_D6_Dc36(prec):
    """Full 16x16, D = 6, Dc = 36 shapes (matrices beyond the LDS: global-memory paths),
    two sampled configurations against the oracle."""
    lat, A, S, _ = make_workload("16x16_D6_Dc36", 2)
    la, sg, fl = _np(*_peps().log_amplitude(*_dev(A, S), lat, prec))
    la_o, sg_o, _ = O.log_amplitude(A, lat, S)
    assert np.all(fl == 0)
    err = np.abs(la - la_o) / np.maximum(1.0, np.abs(la_o))
    _say("16x16 D6 Dc36 %s: max log-amp rel err %.2e (bound %.0e)" % (prec, err.max(), TOL_AMP_16[prec]))
    _assert_amp(la, sg, la_o, sg_o, TOL_AMP_16[prec])


@pytest.mark.xfail(reason="float32 environments move the exchange ratios of about 14% of these "
                          "configurations by more than 1e-4 (the log-amplitudes stay within 1e-5)",
                   strict=False)
def test_float32_local_energy_tail_over_512_samples():
    """Local energies of the first 512 configurations of the 8x8, D = 4, Dc = 16 batch
    in float32 against the float64 path (which matches the oracle to 1e-9 on the tested
    samples), held to the stated 1e-4 bound on every sample, with median / p99 / max
    printed.  The log-amplitudes meet the float32 bound of 1e-5 and the signs agree.
    Running only the sandwich and environment GEMMs in float64 (float32 apply) leaves
    the same tail, so it comes from the float32 environments, not the sandwiches."""
    p = _peps()
    lat, A, S, _ = make_workload("8x8_D4_Dc16", 512)
    Ad, Sd = _dev(A, S)
    la0, sg0, e0, fl0 = _np(*p.local_energy(Ad, Sd, lat, "f64"))
    la, sg, e, fl = _np(*p.local_energy(Ad, Sd, lat, "f32"))
    assert ((fl == 0) & (fl0 == 0)).all()
    err = np.abs(e - e0) / np.maximum(1.0, np.abs(e0))
    ea = np.abs(la - la0) / np.maximum(1.0, np.abs(la0))
    _say("8x8 f32 over 512: E_loc err median %.2e p99 %.2e max %.2e (%d above 1e-4); log-amp max %.2e"
         % (np.median(err), np.quantile(err, 0.99), err.max(), int((err > 1e-4).sum()), ea.max()))
    assert np.array_equal(sg, sg0)
    assert ea.max() <= 1e-5
    assert err.max() <= 1e-4


def test_product_state_24x24_geometry():
    """24x24 open lattice (the largest lattice of the paper's runs) with a random product
    state embedded at D = 2 (Dc = 4, gauge-dressed): closed-form ln|W| and E(S) at any size."""
    import pins_lib as P
    lat = Lattice(24, 24, 2, 4)
    rng = np.random.default_rng(11)
    a = rng.uniform(0.5, 1.5, size=(lat.N, 2)) * rng.choice([-1, 1], size=(lat.N, 2))
    A = P.gauge_dress(P.product_peps(lat, a, rng, 0.3), lat, rng)
    _, S = make_random(lat, 4, 23)
    la, sg, e, fl = _np(*_peps().local_energy(*_dev(A, S), lat, "f64"))
    nn, nnn = P.lattice_bonds(lat.Lx, lat.Ly)
    for b in range(len(S)):
        s = S[b]
        vals = a[np.arange(lat.N), s]
        assert fl[b] == 0
        assert abs(la[b] - np.sum(np.log(np.abs(vals)))) <= 1e-10 * abs(la[b])
        assert sg[b] == int(np.prod(np.sign(vals)))
        sig = 1 - 2 * s.astype(int)
        E = 0.0
        for bonds, J in ((nn, lat.J1), (nnn, lat.J2)):
            for m, n in bonds:
                E += J * sig[m] * sig[n] / 4
                if s[m] != s[n]:
                    E += J * 0.5 * a[m, 1 - s[m]] * a[n, 1 - s[n]] / (a[m, s[m]] * a[n, s[n]])
        assert abs(e[b] - E) <= 1e-9 * max(1.0, abs(E))


def test_eval_jobs_mixed_lattices_graph():
    """Three lattices of different size, D and Dc in one captured HIP graph: every
    job's outputs equal those of a separate evaluation bit for bit, and three replays
    of the cached graph (with eager work in between) reproduce them."""
    p = _peps()
    specs = [("4x4_D2_Dc4", 20, 3), ("8x8_D4_Dc16", 7, 1)]
    jobs, ref = [], []
    for name, B, gm in specs:
        lat, A, S, _ = make_workload(name, B)
        Ad, Sd = _dev(A, S)
        jobs.append({"A": Ad, "S": Sd, "lat": lat, "grad_mode": gm})
        ref.append(_np(*[t for t in p.evaluate(Ad, Sd, lat, "f32", grad_mode=gm)]))
    lat3 = Lattice(6, 5, 3, 9)
    A3, S3 = make_random(lat3, 5, 4)
    A3d, S3d = _dev(A3, S3)
    jobs.append({"A": A3d, "S": S3d, "lat": lat3, "grad_mode": 0})
    la, sg, fl = p.log_amplitude(A3d, S3d, lat3, "f32")
    _, _, e3, _ = p.local_energy(A3d, S3d, lat3, "f32")
    ref.append(_np(la, sg, e3, fl))
    outs = p.eval_jobs(jobs, "f32", graph=True)
    for rep in range(4):
        for k, o in enumerate(outs):
            la, sg, e, g, fl = o
            r = ref[k]
            got = _np(la, sg, e, fl) if g is None else _np(la, sg, e, g, fl)
            want = [r[0], r[1], r[2], r[3]] if g is None else r
            for x, y in zip(got, want):
                assert np.array_equal(x, y, equal_nan=True), (rep, k)
        # clear the outputs, do unrelated eager work, replay the cached graph
        for o in outs:
            for t in o:
                if t is not None:
                    t.zero_()
        torch.cuda.synchronize()
        _ = p.log_amplitude(jobs[0]["A"], jobs[0]["S"], jobs[0]["lat"], "f64")
        torch.cuda.synchronize()
        outs = p.eval_jobs(jobs, "f32", graph=True, outputs=outs)
    # the results of the 4x4 job also match the oracle
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 20)
    la_o, sg_o, e_o, _ = O.local_energy(A, lat, S)
    la, sg, e, _, _ = _np(*outs[0])
    _assert_amp(la, sg, la_o, sg_o, TOL_AMP["f32"])
    _assert_e(e, e_o, TOL_E["f32"])


def test_autotune_keeps_results():
    """The tile autotuner times every candidate tile per GEMM shape; all tiles
    accumulate in the same order, so results after tuning are bitwise unchanged."""
    import os
    import tempfile
    p = _peps()
    lat, A, S, _ = make_workload("8x8_D4_Dc16", 16)
    Ad, Sd = _dev(A, S)
    before = _np(*p.evaluate(Ad, Sd, lat, "f32", grad_mode=3))
    n = p.autotune(Ad, Sd, lat, "f32")
    assert n > 0
    after = _np(*p.evaluate(Ad, Sd, lat, "f32", grad_mode=3))
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tiles.txt")
        p.tune_save(path)
        lines = [ln for ln in open(path) if not ln.startswith("#")]
        assert len(lines) >= n
        p.tune_load(path)


@pytest.mark.parametrize("case", [("8x8_D4_Dc16", "f32"), ("8x8_D4_Dc16", "f64"), ("6x5_D6_Dc36", "f64")])
def test_every_gemm_tile_gives_identical_results(case):
    """Every GEMM tile the autotuner may pick (the matrix-core tiles of each k stage, the
    persistent pipelined forms and the row kernels) sums each output in the same order,
    so forcing one tile onto every GEMM shape of the path leaves all results bit for bit
    equal to those before (tile 0 is the heuristic choice; the loader ignores numbers
    past the last tile)."""
    import os
    import tempfile
    p = _peps()
    name, prec = case
    if name == "6x5_D6_Dc36":
        lat = Lattice(6, 5, 6, 36)
        A, S = make_random(lat, 6, 31, "half")
    else:
        lat, A, S, _ = make_workload(name, 16)
    Ad, Sd = _dev(A, S)
    with tempfile.TemporaryDirectory() as d:
        saved = os.path.join(d, "saved.txt")
        p.tune_save(saved)
        base = _np(*p.evaluate(Ad, Sd, lat, prec, grad_mode=3))
        p.autotune(Ad, Sd, lat, prec)
        path = os.path.join(d, "t.txt")
        p.tune_save(path)
        keys = [ln.split()[0] for ln in open(path) if ln.strip() and not ln.startswith("#")]
        assert keys
        try:
            for t in range(0, 41):
                with open(path, "w") as f:
                    f.writelines(f"{k} {t}\n" for k in keys)
                p.tune_load(path)
                got = _np(*p.evaluate(Ad, Sd, lat, prec, grad_mode=3))
                for nm, x, y in zip(("log-amp", "sign", "E_loc", "grad", "flags"), got, base):
                    assert np.array_equal(x, y), (t, nm)
        finally:
            with open(path, "w") as f:
                f.writelines(f"{k} 0\n" for k in keys)
            p.tune_load(path)
            p.tune_load(saved)


def _eval_form(p, Ad, Sd, lat, fused):
    p.set_fused_steps(fused)
    try:
        return _np(*p.evaluate(Ad, Sd, lat, "f32", grad_mode=1))
    finally:
        p.set_fused_steps(True)


def test_fused_pair_step_matches_gemm_path():
    """The fused sandwich steps accumulate every product in the order of the unfused
    GEMMs (float32 operands, k ascending), so amplitudes, local energies and
    log-derivatives equal those of the GEMM path exactly: each 16x16x4 MFMA sums its four
    products in k order with one rounding per product and the operands are laid out so
    that consecutive MFMAs take consecutive k."""
    p = _peps()
    lat, A, S, _ = make_workload("8x8_D4_Dc16", 37)
    _fused_forms_equal_plain(p, lat, A, S)


@pytest.mark.parametrize("shape", [(4, 4, 2, 4), (5, 4, 3, 9), (3, 6, 4, 11)])
def test_fused_steps_ragged_shapes(shape):
    """The same bitwise agreement where legs (D = 2, 3) and boundary bonds (Dc = 9, 11)
    are below the fused kernels' padded sizes, so bond chunks end part-full, on
    non-square lattices."""
    Lx, Ly, D, Dc = shape
    lat = Lattice(Lx, Ly, D, Dc)
    A, S = make_random(lat, 21, 5 + D)
    _fused_forms_equal_plain(_peps(), lat, A, S)


def _fused_forms_equal_plain(p, lat, A, S):
    Ad, Sd = _dev(A, S)
    p.profile_enable(("fused",))   # counts fused-step launches, so a fallback cannot pass
    try:
        plain = _eval_form(p, Ad, Sd, lat, False)
        assert p.profile_read("fused")[1] == 0
        n0 = p.profile_read("fused")[1]
        fused = _eval_form(p, Ad, Sd, lat, True)
        assert p.profile_read("fused")[1] > n0, "fused steps did not run"
        for name, x, y in zip(("log-amp", "sign", "E_loc", "grad", "flags"), fused, plain):
            d = np.abs(np.asarray(x, np.float64) - np.asarray(y, np.float64))
            assert np.array_equal(x, y), (name, int((d > 0).sum()), d.size, float(d.max()))
    finally:
        p.profile_enable(())


@pytest.mark.parametrize("grad_mode", [2, 3])
def test_gradient_reduction_several_partitions(grad_mode):
    """Eq. (5) sums over a batch of 300 samples, which the library splits into several
    fixed partitions summed in order (the partitioned path the benchmark runs): the
    weighted sum (grad_mode 2) and dE/dA (grad_mode 3) equal the oracle's at 1e-10."""
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 256)
    A2, S2 = make_random(lat, 44, 77, "half")
    S = np.concatenate([S, S2])
    Ad, Sd = _dev(A, S)
    per = O.log_derivative(A, lat, S)
    if grad_mode == 2:
        w = np.random.default_rng(5).standard_normal(len(S))
        g, _, _, _ = _peps().log_derivative(Ad, Sd, lat, "f64", weights=torch.from_numpy(w).cuda())
        (g,) = _np(g)
        ref = np.einsum("b,bnse->nse", w, per)
    else:
        _, _, e, g, fl = _np(*_peps().evaluate(Ad, Sd, lat, "f64", grad_mode=3))
        assert np.all(fl == 0)
        _, _, e_o, _ = O.local_energy(A, lat, S)
        Bn = len(S)
        ref = 2.0 * np.einsum("b,bnse->nse", e_o, per) / Bn - 2.0 * (per.sum(0) / Bn) * e_o.mean()
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    _say("gradient reduction over %d samples, grad_mode %d: rel l2 err %.2e" % (len(S), grad_mode, err))
    assert err <= 1e-10


@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_graded_boundary_spectra_f64(eps):
    """Decaying boundary spectra (the regime of trained states): a random product state
    embedded at D = 4 and gauge-dressed, plus eps times a Gaussian, so the boundary
    singular values fall off by about eps per order.  Log-amplitude, local energy and
    log-derivatives match the oracle at the f64 bounds."""
    import pins_lib as P
    lat = Lattice(8, 8, 4, 16)
    rng = np.random.default_rng(13)
    a = rng.uniform(0.5, 1.5, size=(lat.N, 2)) * rng.choice([-1, 1], size=(lat.N, 2))
    A = P.gauge_dress(P.product_peps(lat, a, rng, 0.0), lat, rng, horizontal=True, vertical="orthogonal")
    A = A + eps * rng.standard_normal(A.shape)
    _, S = make_random(lat, 4, 29)
    la, sg, e, d, fl = _np(*_peps().evaluate(*_dev(A, S), lat, "f64", grad_mode=1))
    for b in range(len(S)):
        la_o, sg_o, e_o, d_o, fl_o = O.full_path_one(A, lat, S[b])
        assert fl[b] == 0 and fl_o == 0 and sg[b] == sg_o
        el = abs(la[b] - la_o) / max(1, abs(la_o))
        ee = abs(e[b] - e_o) / max(1, abs(e_o))
        eg = np.linalg.norm(d[b] - d_o) / np.linalg.norm(d_o)
        _say("graded eps=%g sample %d: log-amp %.2e E_loc %.2e grad %.2e" % (eps, b, el, ee, eg))
        assert el <= TOL_AMP["f64"] and ee <= TOL_E["f64"] and eg <= TOL_G["f64"]


@pytest.mark.parametrize("shape", [(6, 4, 6, 36), (6, 3, 8, 64)])
def test_blocked_qr_shapes_full_path(shape):
    """Column matrices of up to 1296 x 216 (D = 6, Dc = 36) and 4096 x 512 (D = 8, Dc = 64),
    the bulk shapes of the 16x16 and 24x24 lattices, take the blocked QR (register panels,
    matrix-core WY updates) and the WY application of Q: amplitude, local energy and
    log-derivatives equal the oracle at the f64 bounds."""
    Lx, Ly, D, Dc = shape
    lat = Lattice(Lx, Ly, D, Dc)
    A, S = make_random(lat, 3, 40 + D)
    la, sg, e, d, fl = _np(*_peps().evaluate(*_dev(A, S), lat, "f64", grad_mode=1))
    for b in range(len(S)):
        la_o, sg_o, e_o, d_o, fl_o = O.full_path_one(A, lat, S[b])
        assert fl[b] == 0 and fl_o == 0 and sg[b] == sg_o
        el = abs(la[b] - la_o) / max(1, abs(la_o))
        ee = abs(e[b] - e_o) / max(1, abs(e_o))
        eg = np.linalg.norm(d[b] - d_o) / np.linalg.norm(d_o)
        _say("blocked-QR shape %s sample %d: log-amp %.2e E_loc %.2e grad %.2e" % (shape, b, el, ee, eg))
        assert el <= TOL_AMP["f64"] and ee <= TOL_E["f64"] and eg <= TOL_G["f64"]
