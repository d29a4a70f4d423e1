"""Variational boundary compression on the GPU (through the C ABI) against the FP64
oracle with the same sweep count, element by element.

Tolerances as for the SVD truncation in float64 (the compression runs in float64 in
every precision mode): log-amplitude |d| <= 1e-10 max(1, |ln W|) with equal signs,
local energy 1e-9 relative to max(1, |E|), per-sample log-derivative relative l2 1e-9.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1806_03761_amd.workloads import Lattice, make_random, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_AMP, TOL_E, TOL_G = 1e-10, 1e-9, 1e-9


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


@pytest.fixture
def truncation():
    p = _peps()

    def set_(sweeps):
        p.set_truncation(sweeps)

    yield set_
    p.set_truncation(0)


def _eval(A, S, lat, grad_mode=1):
    la, sg, e, g, fl = _peps().evaluate(*_dev(A, S), lat, "f64", grad_mode=grad_mode)
    if grad_mode:
        return _np(la, sg, e, g, fl)
    la, sg, e, fl = _np(la, sg, e, fl)
    return la, sg, e, None, fl


def _check(lat, A, S, sweeps, with_e=True, with_g=True):
    la, sg, e, g, fl = _eval(A, S, lat, 1 if with_g else 0)
    assert np.all(fl == 0), fl
    worst = [0.0, 0.0, 0.0]
    for b in range(len(S)):
        if with_e or with_g:
            la_o, sg_o, e_o, d_o, fl_o = O.full_path_one(A, lat, S[b], sweeps)
        else:
            la_o, sg_o, fl_o = O.log_amplitude_one(A, lat, S[b], sweeps)
        assert fl_o == 0
        assert int(sg[b]) == int(sg_o), (b, sg[b], sg_o)
        ea = abs(la[b] - la_o) / max(1.0, abs(la_o))
        worst[0] = max(worst[0], ea)
        assert ea <= TOL_AMP, f"sample {b}: log-amp error {ea:.3e}"
        if with_e:
            ee = abs(e[b] - e_o) / max(1.0, abs(e_o))
            worst[1] = max(worst[1], ee)
            assert ee <= TOL_E, f"sample {b}: E_loc error {ee:.3e}"
        if with_g:
            eg = np.linalg.norm(g[b] - d_o) / max(np.linalg.norm(d_o), 1e-300)
            worst[2] = max(worst[2], eg)
            assert eg <= TOL_G, f"sample {b}: log-derivative error {eg:.3e}"
    _say(f"  worst errors: amp {worst[0]:.2e} E {worst[1]:.2e} grad {worst[2]:.2e}")
    return la


@pytest.mark.parametrize("lat,seed,scaling", [
    (Lattice(4, 4, 2, 4), 21, "half"), (Lattice(6, 6, 2, 3), 22, "half"), (Lattice(5, 5, 3, 4), 23, "half"),
    (Lattice(7, 4, 3, 5), 24, "frobenius"), (Lattice(4, 6, 2, 2), 25, "half"),
    (Lattice(2, 6, 3, 2), 29, "half"), (Lattice(3, 5, 2, 3), 30, "half")])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_variational_small_lattices(lat, seed, scaling, sweeps, truncation):
    A, S = make_random(lat, 5, seed, scaling)
    _say("variational", lat, "sweeps", sweeps)
    truncation(sweeps)
    _check(lat, A, S, sweeps)


def test_variational_changes_w_only_where_truncating(truncation):
    """The SVD and variational truncations agree in the exact regime (4x4, D2, Dc4) and
    differ in the truncated one (6x6, D2, Dc3)."""
    for lat, differ in ((Lattice(4, 4, 2, 4), False), (Lattice(6, 6, 2, 3), True)):
        A, S = make_random(lat, 6, 26, "half")
        truncation(0)
        l0 = _eval(A, S, lat, 0)[0]
        truncation(1)
        l1 = _eval(A, S, lat, 0)[0]
        d = np.max(np.abs(l1 - l0))
        _say("variational vs svd", lat, f"{d:.2e}")
        assert (d > 1e-6) if differ else (d < 1e-10)


def test_variational_8x8_D4_Dc16(truncation):
    lat, A, S, _ = make_workload("8x8_D4_Dc16", 6)
    _say("variational 8x8 D4 Dc16")
    truncation(1)
    _check(lat, A, S, 1)


def _oracle_noise(A, lat, s, sweeps, la, seeds=(1, 2)):
    """The oracle's own rounding noise on ln|W|: W is linear in every site tensor (the
    compression is homogeneous in the applied row), so scaling site m by 1 + d_m
    (|d_m| <= 2^-30) moves ln|W| by exactly sum ln(1 + d_m); whatever else moves is
    rounding.  Relative to max(1, |ln W|), the largest over the seeds."""
    worst = 0.0
    for k in seeds:
        d = np.random.default_rng(7100 + k).uniform(-1.0, 1.0, size=lat.N) * 2.0 ** -30
        la2 = O.log_amplitude_one(A * (1.0 + d)[:, None, None, None, None, None], lat, s, sweeps)[0]
        worst = max(worst, abs(la2 - float(np.sum(np.log1p(d))) - la) / max(1.0, abs(la)))
    return worst


def test_variational_16x16_D6_Dc36_amplitude(truncation):
    """At 16x16, D = 6, Dc = 36 one sweep passes rounding on from row to row (each
    boundary is linear in its guess, the previous boundary), so the oracle's own noise
    on ln|W| reaches ~1e-10 (1e-12 with the SVD truncation): the bound is 10x that noise,
    measured on the oracle alone, and never below 1e-10."""
    lat, A, S, _ = make_workload("16x16_D6_Dc36", 2)
    _say("variational 16x16 D6 Dc36 amplitude")
    truncation(1)
    la, sg, _, _, fl = _eval(A, S, lat, 0)
    assert np.all(fl == 0)
    for b in range(len(S)):
        la_o, sg_o, fl_o = O.log_amplitude_one(A, lat, S[b], 1)
        assert fl_o == 0 and int(sg[b]) == int(sg_o)
        noise = _oracle_noise(A, lat, S[b], 1, la_o)
        err = abs(la[b] - la_o) / max(1.0, abs(la_o))
        _say(f"  sample {b}: error {err:.2e}, oracle noise {noise:.2e}")
        assert err <= max(TOL_AMP, 10.0 * noise)


def test_variational_D16_Dc32(truncation):
    """The Dc = 2D regime at D = 16 (4x4 lattice): amplitude, local energy and
    log-derivative."""
    lat = Lattice(4, 4, 16, 32)
    A, S = make_random(lat, 2, 27)
    _say("variational 4x4 D16 Dc32")
    truncation(1)
    _check(lat, A, S, 1)


def test_variational_chunked_equals_single_chunk(truncation):
    """A workspace limit that splits the batch into chunks gives the same bits."""
    p = _peps()
    lat = Lattice(6, 6, 3, 5)
    A, S = make_random(lat, 40, 28)
    truncation(2)
    ref = _eval(A, S, lat)
    try:
        p.set_workspace_limit(p.workspace_bytes(lat, 7))
        got = _eval(A, S, lat)
    finally:
        p.set_workspace_limit(0)
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)


GOLD = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _golden(name, kind, b):
    import json
    import os
    path = os.path.join(GOLD, f"var_{name}_{kind}_{b}.json")
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} not generated")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["mix_16x16_D8_Dc64"])
def test_variational_D8_Dc64_against_goldens(name, truncation):
    """D = 8, Dc = 64 (the 16x16 lattice of the uneven batch): the site factorisations
    (512 x 64) run from global scratch.  Stored oracle values
    (tests/golden/make_goldens_variational.py), each with the oracle's own rounding noise:
    ln|W| within max(1e-10 |ln W|, 10 noise), E(S) within max(1e-9 max(1, |E|), 10 noise).
    (At 24x24 the same truncation amplifies rounding about fourfold per row: the oracle's
    noise on ln|W| is 0.1-0.3 there, so its stored values bound nothing useful.)"""
    g0 = _golden(name, "amp", 0)
    lat, A, S, _ = make_workload(name, 2)
    _say("variational", name)
    truncation(1)
    la, sg, fl = _np(*_peps().log_amplitude(*_dev(A, S), lat, "f64"))
    assert np.all(fl == 0), fl
    for b in range(2):
        g = g0 if b == 0 else _golden(name, "amp", 1)
        assert g["config"] == S[b].tolist()
        err = abs(la[b] - g["log_abs"])
        _say(f"  sample {b}: |d ln W| {err:.2e}, oracle noise {g['noise']:.2e}")
        assert int(sg[b]) == g["sign"]
        assert err <= max(TOL_AMP * abs(g["log_abs"]), 10.0 * g["noise"])
    import os
    if os.path.exists(os.path.join(GOLD, f"var_{name}_eloc_0.json")):
        ge = _golden(name, "eloc", 0)
        e = _eval(A[:], S[:1], lat, 0)[2]
        err = abs(e[0] - ge["e_loc"])
        _say(f"  sample 0: |d E| {err:.2e}, oracle noise {ge['noise']:.2e}")
        assert err <= max(TOL_E * max(1.0, abs(ge["e_loc"])), 10.0 * ge["noise"])


def test_variational_in_a_captured_graph(truncation):
    """Two lattices with variational compression in one captured HIP graph: each job's
    outputs equal a separate evaluation bit for bit, over three replays with eager work in
    between; switching the truncation back captures a new graph (the cached one is keyed
    on it) whose results equal the SVD truncation's."""
    p = _peps()
    specs = [(Lattice(6, 6, 2, 3), 9, 41), (Lattice(5, 7, 3, 4), 6, 42)]
    truncation(1)
    jobs, ref = [], []
    for lat, B, seed in specs:
        A, S = make_random(lat, B, seed, "half")
        Ad, Sd = _dev(A, S)
        jobs.append({"A": Ad, "S": Sd, "lat": lat, "grad_mode": 1})
        ref.append(_np(*p.evaluate(Ad, Sd, lat, "f64", grad_mode=1)))
    outs = p.eval_jobs(jobs, "f64", graph=True)
    for rep in range(3):
        for k, o in enumerate(outs):
            for x, y in zip(_np(*o), ref[k]):
                assert np.array_equal(x, y, equal_nan=True), (rep, k)
        for o in outs:
            for t in o:
                t.zero_()
        torch.cuda.synchronize()
        _ = p.log_amplitude(jobs[0]["A"], jobs[0]["S"], jobs[0]["lat"], "f64")
        torch.cuda.synchronize()
        outs = p.eval_jobs(jobs, "f64", graph=True, outputs=outs)
    truncation(0)
    svd = _np(*p.evaluate(jobs[0]["A"], jobs[0]["S"], jobs[0]["lat"], "f64", grad_mode=1))
    outs = p.eval_jobs(jobs, "f64", graph=True, outputs=outs)
    for x, y in zip(_np(*outs[0]), svd):
        assert np.array_equal(x, y, equal_nan=True)
    assert not np.array_equal(svd[0], ref[0][0])


def test_variational_register_factorisation_ragged(truncation):
    """6x6, D = 7, Dc = 60: the middle sites factorise 343 x 60 and 420 x 49 matrices, too
    large for LDS and not multiples of the wave width, so they take the register-resident
    thin QR: amplitudes, local energies and log-derivatives against the oracle."""
    lat = Lattice(6, 6, 7, 60)
    A, S = make_random(lat, 2, 43)
    _say("variational 6x6 D7 Dc60 (register factorisation)")
    truncation(1)
    _check(lat, A, S, 1)


def test_variational_global_scratch_factorisation(truncation):
    """6x5, D = 12, Dc = 70: the middle sites factorise 840 x 70 matrices (470 KB), beyond
    the register and LDS forms, so the thin QR works in global scratch: amplitudes
    against the oracle."""
    lat = Lattice(6, 5, 12, 70)
    A, S = make_random(lat, 2, 45)
    _say("variational 6x5 D12 Dc70 (global-scratch factorisation)")
    truncation(1)
    _check(lat, A, S, 1, with_e=False, with_g=False)


def test_variational_dc_three_d(truncation):
    """The Dc = 3D case of the Dc proportional to D regime (5x5, D = 8, Dc = 24):
    amplitudes, local energies and log-derivatives against the oracle."""
    lat = Lattice(5, 5, 8, 24)
    A, S = make_random(lat, 3, 44)
    _say("variational 5x5 D8 Dc24")
    truncation(1)
    _check(lat, A, S, 1)


def test_variational_metropolis_matches_oracle(truncation):
    """The sampler contracts W(S') with the context's truncation: four Metropolis steps of
    24 chains on 6x6, D = 2, Dc = 3 with variational compression take the oracle's moves
    (same uniforms), with ln|W| to 1e-10; a decision may differ only inside the rounding
    band of its margin |2 (ln|W(S')| - ln|W(S)|) - ln u|, and such a chain is dropped."""
    p = _peps()
    lat = Lattice(6, 6, 2, 3)
    A, S0 = make_random(lat, 24, 47, "half")
    U = np.random.default_rng(48).random((4, S0.shape[0], 2))
    truncation(1)
    Ad, Sd = _dev(A, S0)
    la_d, sg_d, _ = p.log_amplitude(Ad, Sd, lat, "f64")
    la_o, sg_o, fl_o = O.log_amplitude(A, lat, S0, 1)
    assert np.all(fl_o == 0)
    So = S0.copy()
    live = np.ones(S0.shape[0], dtype=bool)
    bonds = O.proposal_bonds(lat)
    nb = len(bonds)
    moves = 0
    for t in range(4):
        acc_d = p.metropolis_step(Ad, Sd, lat, torch.from_numpy(U[t]).cuda(), la_d, sg_d, "f64")
        S_g, la_g, sg_g, acc_g = _np(Sd, la_d, sg_d, acc_d)
        So_new, la_new, sg_new, acc_o = O.metropolis_step(A, lat, So, U[t], la_o, sg_o, sweeps=1)
        for b in range(S0.shape[0]):
            if not live[b]:
                continue
            if bool(acc_o[b]) != bool(acc_g[b]):
                m, n = bonds[min(int(U[t, b, 0] * nb), nb - 1)]
                Sp = So[b].copy()
                Sp[m], Sp[n] = So[b, n], So[b, m]
                lap = O.log_amplitude_one(A, lat, Sp, 1)[0]
                margin = abs(2.0 * (lap - la_o[b]) - np.log(U[t, b, 1]))
                assert margin <= 4.0 * TOL_AMP * max(1.0, abs(lap)), (t, b, margin)
                live[b] = False
                continue
            assert np.array_equal(So_new[b], S_g[b]) and sg_new[b] == sg_g[b], (t, b)
            assert abs(la_new[b] - la_g[b]) <= TOL_AMP * max(1.0, abs(la_new[b])), (t, b)
            moves += int(acc_g[b])
        So, la_o, sg_o = So_new, la_new, sg_new
    _say(f"  accepted moves compared: {moves}, chains kept {int(live.sum())}")
    assert moves > 0 and live.sum() >= S0.shape[0] - 2


def test_variational_pair_correlations_match_oracle(truncation):
    """Spin-spin correlations contract every exchanged configuration with the context's
    truncation: 6x6, D = 2, Dc = 3, variational compression, the centre site with every
    site, per-sample values and means to 1e-10."""
    p = _peps()
    lat = Lattice(6, 6, 2, 3)
    A, S = make_random(lat, 8, 49, "half")
    pairs = [(14, m) for m in range(lat.N)]
    truncation(1)
    means, vals, fl = p.pair_correlations(*_dev(A, S), lat, pairs, "f64", per_sample=True)
    means, vals, fl = _np(means, vals, fl)
    m_o, v_o, fl_o = O.pair_correlations(A, lat, S, pairs, sweeps=1)
    assert np.array_equal(fl, fl_o) and np.all(fl_o == 0)
    err = np.abs(vals - v_o) / np.maximum(1.0, np.abs(v_o))
    assert err.max() <= 1e-10, err.max()
    assert np.max(np.abs(means - m_o) / np.maximum(1.0, np.abs(m_o))) <= 1e-10
