"""Spin-spin correlations and the structure factor on the GPU (peps_pair_correlations,
peps_structure_factor, through the C ABI) against the FP64 oracle.

Tolerances on a local value v = sigma sigma / 4 + ratio / 2: f64 1e-10, f32 2e-4, relative
to max(1, |v|) (the ratio carries the error of two log-amplitudes, each within the
amplitude tolerance, exponentiated).  Means: the same bounds.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1806_03761_amd.workloads import Lattice, make_random, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 2e-4}


def _peps():
    from paper_1806_03761_amd import peps
    return peps


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _close(a, b, tol):
    both_nan = np.isnan(a) & np.isnan(b)
    err = np.where(both_nan, 0.0, np.abs(a - b) / np.maximum(1.0, np.abs(b)))
    assert not np.isnan(err).any(), "NaN pattern differs"
    assert err.max() <= tol, f"max error {err.max():.3e} > {tol}"


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_pair_correlations_4x4(prec):
    """4x4 D2 Dc4: 40 samples (one with a spin value outside {0, 1}, which is left out),
    pairs of the centre site with every site (itself included) and a few long ones."""
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 40)
    S = S.copy()
    S[7, 3] = 2
    pairs = [(5, m) for m in range(lat.N)] + [(0, 15), (3, 12), (12, 3), (6, 9)]
    _say("4x4 pair correlations", prec, len(pairs), "pairs")
    means, vals, fl = _peps().pair_correlations(_cuda(A), _cuda(S), lat, pairs, prec, per_sample=True)
    torch.cuda.synchronize()
    m_o, v_o, fl_o = O.pair_correlations(A, lat, S, pairs)
    assert np.array_equal(fl.cpu().numpy(), fl_o)
    assert fl_o[7] == O.FLAG_BAD_CONFIG
    _close(vals.cpu().numpy(), v_o, TOL[prec])
    _close(means.cpu().numpy(), m_o, TOL[prec])
    assert np.all(vals.cpu().numpy()[fl_o == 0, 5] == 0.75)


def test_structure_factor_matches_oracle():
    """Seeded symmetric correlation matrices over the central block of 8x8 and a ragged
    3x5 block; k on a grid including (pi, pi) and (0, 0)."""
    rng = np.random.default_rng(5)
    for lat, sites in ((Lattice(8, 8, 4, 16), O.bulk_sites(Lattice(8, 8, 4, 16))),
                       (Lattice(3, 5, 2, 4), [1, 4, 7, 10, 13, 2, 8])):
        n = len(sites)
        C = rng.standard_normal((n, n))
        C = 0.5 * (C + C.T)
        ks = [(np.pi, np.pi), (0.0, 0.0), (np.pi, 0.0), (0.3, -1.1), (2.5, 0.7)]
        _say("structure factor", n, "sites")
        got = _peps().structure_factor(_cuda(C), lat, sites, ks).cpu().numpy()
        want = O.structure_factor(lat, sites, C, ks)
        assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max())


def test_correlations_and_m2_4x4_end_to_end():
    """4x4 D2 Dc4, 24 samples: the correlation matrix of the central 2x2 block ((L - 2) x
    (L - 2) of a 4x4 lattice, margin 1) and m^2 at (pi, pi) and (0, 0), f64."""
    peps = _peps()
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 24)
    sites = O.bulk_sites(lat, margin=1)
    C, fl = peps.correlation_matrix(_cuda(A), _cuda(S), lat, sites, "f64")
    ks = [(np.pi, np.pi), (0.0, 0.0)]
    m2 = peps.structure_factor(C, lat, sites, ks).cpu().numpy()
    pairs = [(a, b) for a in sites for b in sites]
    m_o, _, fl_o = O.pair_correlations(A, lat, S, pairs)
    C_o = m_o.reshape(len(sites), len(sites))
    _close(C.cpu().numpy(), C_o, 1e-10)
    _close(m2, O.structure_factor(lat, sites, C_o, ks), 1e-10)


def test_pair_correlations_8x8_full_batch_sampled():
    """8x8 D4 Dc16 with 4096 samples, f32: the (L-4) x (L-4) central block's 136 pairs
    (i <= j); per-sample values of three samples (first, last, one between) against the
    oracle, every sample's diagonal entries 3/4 and the matrix of means symmetric in use."""
    peps = _peps()
    lat, A, S, _ = make_workload("8x8_D4_Dc16")
    sites = O.bulk_sites(lat)
    pairs = [(sites[a], sites[b]) for a in range(len(sites)) for b in range(a, len(sites))]
    _say("8x8 correlations, 4096 samples,", len(pairs), "pairs")
    means, vals, fl = peps.pair_correlations(_cuda(A), _cuda(S), lat, pairs, "f32", per_sample=True)
    torch.cuda.synchronize()
    vals = vals.cpu().numpy()
    assert np.all(fl.cpu().numpy() == 0)
    check = [0, 1711, S.shape[0] - 1]
    _, v_o, fl_o = O.pair_correlations(A, lat, S[check], pairs)
    assert np.all(fl_o == 0)
    _close(vals[check], v_o, TOL["f32"])
    diag = [k for k, (a, b) in enumerate(pairs) if a == b]
    assert np.all(vals[:, diag] == 0.75)
    m = means.cpu().numpy()
    assert np.abs(m - vals.mean(0)).max() <= 1e-12 * max(1.0, np.abs(m).max())


def test_pair_correlations_rejects_bad_sites():
    peps = _peps()
    lat = Lattice(3, 5, 2, 4)
    A, S = make_random(lat, 4, 3)
    with pytest.raises(peps.PepsError):
        peps.pair_correlations(_cuda(A), _cuda(S), lat, [(0, 15)])
    with pytest.raises(peps.PepsError):
        peps.structure_factor(torch.zeros((1, 1), dtype=torch.float64, device="cuda"), lat, [-1], [(0.0, 0.0)])
