"""Pins of the oracle's variational boundary compression (the truncation alternative
of Sec. II-A whose cost is O(D^4 Dc^2) per site and sweep).

The compression is one-site alternating least squares; its results are fixed by
properties any correct implementation has, each checked with independent dense code:
  * a guess whose bonds span the whole Hilbert space reproduces the state exactly;
  * after every sweep the result is an orthogonal projection of the target
    (<C|P> = <C|C>) and the error never grows from one sweep to the next;
  * on two sites the iteration converges to the best rank-t approximation
    (Eckart-Young, from a dense SVD);
  * a target that already lies in the guess's manifold is returned unchanged;
  * whole-lattice closed forms where the boundary has Schmidt rank one (product
    states; PEPS whose tensors factor into a horizontal and a vertical part), and
    the invariance of W under gauges on horizontal bonds.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.peps_oracle as OP
import pins_lib as P
from paper_1806_03761_amd.workloads import Lattice, make_random


def _rand_mps(rng, bonds, p):
    return [rng.standard_normal((bonds[j], p, bonds[j + 1])) for j in range(len(bonds) - 1)]


def _dense(mps, ln=0.0):
    return P.mps_to_dense(mps).ravel() * math.exp(ln)


def test_full_bond_guess_is_exact():
    """Bonds equal to the full dims min(p^j, p^(n-j)): the right isometries are unitary,
    so the first update already holds the whole state."""
    rng = np.random.default_rng(11)
    p, n = 2, 6
    full = [min(p ** j, p ** (n - j)) for j in range(n + 1)]
    Pm = _rand_mps(rng, [1, 3, 5, 7, 5, 3, 1], p)
    G = _rand_mps(rng, full, p)
    for sweeps in (1, 2):
        C, ln = O.compress_variational(Pm, G, sweeps)
        assert [c.shape[0] for c in C] + [1] == full
        v, w = _dense(C, ln), _dense(Pm)
        assert np.linalg.norm(v - w) < 1e-12 * np.linalg.norm(w)


@pytest.mark.parametrize("p,bondP,bondG", [(2, 6, 3), (3, 5, 4)])
def test_projection_identity_and_monotone_error(p, bondP, bondG):
    """<C|P> = <C|C> after every sweep (the result is the orthogonal projection of P on
    the tangent space of its last update), hence ||P - C||^2 = ||P||^2 - ||C||^2, and the
    error does not grow from sweep to sweep."""
    rng = np.random.default_rng(12 + p)
    n = 6
    bP = [1] + [min(bondP, p ** j, p ** (n - j)) for j in range(1, n)] + [1]
    bG = [1] + [min(bondG, p ** j, p ** (n - j)) for j in range(1, n)] + [1]
    Pm = _rand_mps(rng, bP, p)
    G = _rand_mps(rng, bG, p)
    w = _dense(Pm)
    errs = []
    for sweeps in range(1, 7):
        C, ln = O.compress_variational(Pm, G, sweeps)
        v = _dense(C, ln)
        cc, cp = float(v @ v), float(v @ w)
        assert abs(cp - cc) < 1e-12 * float(w @ w)
        err2 = float((w - v) @ (w - v))
        assert abs(err2 - (float(w @ w) - cc)) < 1e-11 * float(w @ w)
        errs.append(err2)
    assert errs[-1] > 1e-6 * float(w @ w)          # a real truncation
    for a, b in zip(errs, errs[1:]):
        assert b <= a * (1 + 1e-12) + 1e-14


def test_two_sites_converge_to_eckart_young():
    """Two sites: the sweeps are an orthogonal iteration and reach the best rank-2
    approximation of the 4 x 4 matrix (singular values 4, 3, 1, 0.5)."""
    rng = np.random.default_rng(13)
    U, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    V, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    s = np.array([4.0, 3.0, 1.0, 0.5])
    M = U @ np.diag(s) @ V.T
    Pm = [(U * s).reshape(1, 4, 4), V.T.reshape(4, 4, 1)]
    G = _rand_mps(rng, [1, 2, 1], 4)
    C, ln = O.compress_variational(Pm, G, 40)
    Cd = _dense(C, ln).reshape(4, 4)
    best = (U[:, :2] * s[:2]) @ V[:, :2].T
    assert np.linalg.norm(Cd - best) < 1e-10 * np.linalg.norm(M)
    assert abs(np.linalg.norm(M - Cd) ** 2 - 1.25) < 1e-10


def test_state_in_the_guess_manifold_is_kept():
    """Identity row (T[l,u,r,d] = [l = r = 0][u = d]): Apply(E) = E, the guess, so one
    sweep returns the same state."""
    rng = np.random.default_rng(14)
    p, n = 3, 5
    E = _rand_mps(rng, [1, 3, 5, 5, 3, 1], p)
    row = []
    for _ in range(n):
        T = np.zeros((1, p, 1, p))
        T[0, :, 0, :] = np.eye(p)
        row.append(T)
    Pm = O.apply_row_down(E, row)
    assert O.truncated_bonds(Pm, 5) == [1, 3, 5, 5, 3, 1]
    C, ln = O.next_boundary(E, Pm, 5, sweeps=1)
    v, w = _dense(C, ln), _dense(E)
    assert np.linalg.norm(v - w) < 1e-12 * np.linalg.norm(w)


def _count_variational(monkeypatch):
    calls = []
    real = OP.compress_variational

    def counted(Pm, G, sweeps):
        calls.append(sweeps)
        return real(Pm, G, sweeps)

    monkeypatch.setattr(OP, "compress_variational", counted)
    return calls


def _factored_peps(lat, rng):
    """T^s_ij[l,u,r,d] = a^s_ij[l,r] b^s_ij[u,d]: the PEPS is a product of independent
    row chains (a) and column chains (b), so every boundary has Schmidt rank one and W
    is the product of the chain values."""
    D = lat.D
    a = rng.uniform(0.5, 1.5, size=(lat.N, 2, D, D)) * rng.choice([-1, 1], size=(lat.N, 2, D, D))
    b = rng.uniform(0.5, 1.5, size=(lat.N, 2, D, D)) * rng.choice([-1, 1], size=(lat.N, 2, D, D))
    A = np.einsum("msLR,msUD->msLURD", a, b)
    return A, a, b


def _factored_w(lat, a, b, s):
    """(ln|W|, sign W) of the factored PEPS from its chains (outward legs at index 0)."""
    w_log, w_sg = 0.0, 1
    for i in range(lat.Ly):
        v = np.zeros(lat.D)
        v[0] = 1.0
        for j in range(lat.Lx):
            m = i * lat.Lx + j
            v = v @ a[m, s[m]]
        x = v[0]
        w_log += math.log(abs(x))
        w_sg *= int(np.sign(x))
    for j in range(lat.Lx):
        v = np.zeros(lat.D)
        v[0] = 1.0
        for i in range(lat.Ly):
            m = i * lat.Lx + j
            v = v @ b[m, s[m]]
        x = v[0]
        w_log += math.log(abs(x))
        w_sg *= int(np.sign(x))
    return w_log, w_sg


@pytest.mark.parametrize("lat", [Lattice(5, 5, 3, 2), Lattice(6, 4, 2, 3)])
def test_rank_one_boundaries_closed_form(lat, monkeypatch):
    """Factored PEPS (rank-one boundaries): ln|W|, sign and E(S) equal the closed form
    from the chains, with the variational compression engaged on the later rows."""
    calls = _count_variational(monkeypatch)
    rng = np.random.default_rng(15)
    A, a, b = _factored_peps(lat, rng)
    _, S = make_random(lat, 3, 17)
    for sweeps in (1, 2):
        calls.clear()
        la, sg, e, fl = O.local_energy(A, lat, S, sweeps=sweeps)
        assert len(calls) > 0
        for k in range(len(S)):
            s = S[k]
            l0, g0 = _factored_w(lat, a, b, s)
            assert abs(la[k] - l0) < 1e-10 * max(1.0, abs(l0)) and sg[k] == g0
            sig = 1 - 2 * s.astype(int)
            E = 0.0
            nn, nnn = P.lattice_bonds(lat.Lx, lat.Ly)
            for bonds, J in ((nn, lat.J1), (nnn, lat.J2)):
                for m, n in bonds:
                    E += J * sig[m] * sig[n] / 4
                    if s[m] != s[n]:
                        sp = s.copy()
                        sp[m], sp[n] = s[n], s[m]
                        l1, g1 = _factored_w(lat, a, b, sp)
                        E += J * 0.5 * g1 * g0 * math.exp(l1 - l0)
            assert abs(e[k] - E) < 1e-9 * max(1.0, abs(E))


def test_product_state_closed_form_variational(monkeypatch):
    """Gauge-dressed D = 1 product state: ln|W| = sum ln|a_m(s_m)| with the sweeps on."""
    calls = _count_variational(monkeypatch)
    lat = Lattice(5, 4, 3, 2)
    rng = np.random.default_rng(16)
    a = rng.uniform(0.5, 1.5, size=(lat.N, 2)) * rng.choice([-1, 1], size=(lat.N, 2))
    A = P.gauge_dress(P.product_peps(lat, a, rng, 0.3), lat, rng)
    _, S = make_random(lat, 3, 18)
    la, sg, fl = O.log_amplitude(A, lat, S, sweeps=2)
    assert len(calls) > 0
    for k in range(len(S)):
        vals = a[np.arange(lat.N), S[k]]
        assert abs(la[k] - float(np.sum(np.log(np.abs(vals))))) < 1e-11
        assert sg[k] == int(np.prod(np.sign(vals)))


def test_variational_gauge_invariance(monkeypatch):
    """The compression acts on boundary states (guess and target), so invertible gauges
    on horizontal bonds leave W and E unchanged.  (A vertical gauge rotates the target's
    physical legs but not the guess's, which live one row higher, so the sweeps start
    from a different state there: that case is not invariant.)"""
    calls = _count_variational(monkeypatch)
    lat = Lattice(6, 5, 3, 4)
    A, S = make_random(lat, 2, 61)
    la, sg, e, _ = O.local_energy(A, lat, S, sweeps=2)
    assert len(calls) > 0
    A2 = P.gauge_dress(A, lat, np.random.default_rng(1), horizontal=True, vertical=None)
    la2, sg2, e2, _ = O.local_energy(A2, lat, S, sweeps=2)
    assert np.allclose(la2, la, rtol=1e-10, atol=1e-10) and np.all(sg2 == sg)
    assert np.allclose(e2, e, rtol=1e-8, atol=1e-8)


def test_variational_differs_from_svd_and_approaches_it():
    """In the truncated regime the two truncations give different W; more sweeps move
    the variational one no further from the SVD one than a single sweep."""
    lat = Lattice(6, 6, 2, 3)
    A, S = make_random(lat, 4, 5, "half")
    l0 = O.log_amplitude(A, lat, S)[0]
    l1 = O.log_amplitude(A, lat, S, sweeps=1)[0]
    l4 = O.log_amplitude(A, lat, S, sweeps=4)[0]
    assert np.max(np.abs(l1 - l0)) > 1e-6
    assert np.max(np.abs(l4 - l0)) < 0.2


def test_variational_accuracy_weakly_entangled():
    """Against the exact W (the same lattice contracted with Dc at the full boundary rank),
    one sweep is as accurate as the SVD truncation on a weakly entangled state (a product
    state plus half a Gaussian PEPS): both within 1e-6 of ln|W|."""
    lat, latx = Lattice(8, 6, 2, 4), Lattice(8, 6, 2, 16)
    A, S = make_random(lat, 8, 31)
    a = np.random.default_rng(0).uniform(0.5, 1.5, size=(lat.N, 2))
    A2 = 0.5 * A / np.max(np.abs(A))
    A2[:, :, 0, 0, 0, 0] += a
    ex = O.log_amplitude(A2, latx, S)[0]
    for sweeps in (0, 1):
        d = np.abs(O.log_amplitude(A2, lat, S, sweeps)[0] - ex)
        assert d.max() < 1e-6, (sweeps, d.max())
