"""Independent reference computations used to pin the oracle (CPU, float64).

Nothing here is imported from the oracle: every routine is a separate dense
formulation that reaches the same numbers by another route.
  * dense_psi: exact transfer-matrix contraction of the single-layer network
    (Eq. (1) at fixed S) with no MPS and no truncation;
  * dense_psi_truncated: the truncated boundary contraction done on the dense
    boundary vector, projecting every cut onto its leading Schmidt vectors;
  * dense_env_down / dense_env_up / dense_local_energy: the truncated upper and lower
    environments as dense vectors, and the local energy from dense sandwiches of them;
  * full_wavefunction: all 2^N amplitudes of a small PEPS at once;
  * heisenberg_j1j2: the sparse J1-J2 Hamiltonian (Sec. III-A) built from bit
    operations, for brute-force local energies and exact diagonalisation.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def _dims(lat, i, j):
    D = lat.D
    return (1 if j == 0 else D, 1 if i == 0 else D,
            1 if j == lat.Lx - 1 else D, 1 if i == lat.Ly - 1 else D)


def _T(A, lat, i, j, s):
    dl, du, dr, dd = _dims(lat, i, j)
    return A[i * lat.Lx + j, s, :dl, :du, :dr, :dd]


def _push_row(psi, A, lat, S, i):
    """psi over the u-legs of row i (shape (Du,)*Lx) -> vector over its d-legs."""
    Lx = lat.Lx
    X = psi.reshape(1, -1, 1)            # [done d-legs, remaining u-legs, horizontal bond]
    rem = [psi.shape[j] for j in range(Lx)]
    done = []
    for j in range(Lx):
        T = _T(A, lat, i, j, int(S[i * Lx + j]))
        Pd = X.shape[0]
        u = rem[j]
        R = int(np.prod(rem[j + 1:])) if j + 1 < Lx else 1
        H = X.shape[2]
        X4 = X.reshape(Pd, u, R, H)
        Y = np.einsum("puRh,hurd->pdRr", X4, T)
        done.append(T.shape[3])
        X = Y.reshape(Pd * T.shape[3], R, T.shape[2])
    return X.reshape(done)


def dense_psi(A, lat, S):
    """Exact W(S): a dense boundary vector pushed through every row."""
    psi = np.ones([1] * lat.Lx)
    for i in range(lat.Ly):
        psi = _push_row(psi, A, lat, S, i)
    return float(psi.reshape(-1)[0])


def _project_cuts(psi, Dc):
    """Project the dense boundary state onto its leading Dc Schmidt vectors at every
    cut, from the last cut to the first, each projection acting on the current state."""
    shape = psi.shape
    n = len(shape)
    v = psi.reshape(-1)
    for c in range(n - 1, 0, -1):
        left = int(np.prod(shape[:c]))
        M = v.reshape(left, -1)
        _, _, Vt = np.linalg.svd(M, full_matrices=False)
        t = min(Dc, Vt.shape[0])
        Vk = Vt[:t]
        M = (M @ Vk.T) @ Vk
        v = M.reshape(-1)
    return v.reshape(shape)


def dense_psi_truncated(A, lat, S):
    """(sign, ln|W|) of the top-down contraction truncated to Dc, done densely."""
    psi = np.ones([1] * lat.Lx)
    logscale = 0.0
    for i in range(lat.Ly - 1):
        psi = _push_row(psi, A, lat, S, i)
        psi = _project_cuts(psi, lat.Dc)
        nu = np.linalg.norm(psi)
        psi = psi / nu
        logscale += math.log(nu)
    w = float(_push_row(psi, A, lat, S, lat.Ly - 1).reshape(-1)[0])
    return int(np.sign(w)), logscale + math.log(abs(w))


def dense_env_down(A, lat, S, i_stop):
    """Dense truncated upper environment of row i_stop (state over its u-legs), with log."""
    psi = np.ones([1] * lat.Lx)
    logscale = 0.0
    for i in range(i_stop):
        psi = _push_row(psi, A, lat, S, i)
        psi = _project_cuts(psi, lat.Dc)
        nu = np.linalg.norm(psi)
        psi = psi / nu
        logscale += math.log(nu)
    return psi, logscale


def _push_row_up(phi, A, lat, S, i):
    """phi over the d-legs of row i (shape (Dd,)*Lx) -> vector over its u-legs: the row
    is read with u and d exchanged, so the same left-to-right pass applies."""
    Lx = lat.Lx
    X = phi.reshape(1, -1, 1)
    rem = [phi.shape[j] for j in range(Lx)]
    done = []
    for j in range(Lx):
        T = _T(A, lat, i, j, int(S[i * Lx + j])).transpose(0, 3, 2, 1)   # [l, d, r, u]
        Pd = X.shape[0]
        R = int(np.prod(rem[j + 1:])) if j + 1 < Lx else 1
        X4 = X.reshape(Pd, rem[j], R, X.shape[2])
        Y = np.einsum("pdRh,hdru->puRr", X4, T)
        done.append(T.shape[3])
        X = Y.reshape(Pd * T.shape[3], R, T.shape[2])
    return X.reshape(done)


def dense_env_up(A, lat, S, i_stop):
    """Dense truncated lower environment of row i_stop (state over its d-legs), with log:
    rows Ly-1 .. i_stop+1 pushed upwards, each followed by the same cut projection as
    the downward sweep (last cut first) and a normalisation."""
    phi = np.ones([1] * lat.Lx)
    logscale = 0.0
    for i in range(lat.Ly - 1, i_stop, -1):
        phi = _push_row_up(phi, A, lat, S, i)
        phi = _project_cuts(phi, lat.Dc)
        nu = np.linalg.norm(phi)
        phi = phi / nu
        logscale += math.log(nu)
    return phi, logscale


def dense_two_row_sandwich(Udense, A, lat, S, i, Ldense):
    """<U| rows i, i+1 |L> with U over the u-legs of row i and L over the d-legs of row i+1."""
    out = _push_row(_push_row(Udense, A, lat, S, i), A, lat, S, i + 1)
    return float(np.sum(out * Ldense))


def dense_local_energy(A, lat, S, ratio_source="sandwich"):
    """E(S) of Eq. (4) with every exchange ratio from dense sandwiches of the dense
    truncated environments: <U_i|row i|L_i> for a bond inside row i, <U_i|rows i,
    i+1|L_{i+1}> for a bond between rows i and i+1 (numerator and denominator from the
    same sandwich).  ratio_source="full" takes every ratio from the top-down truncated
    contraction of the whole lattice instead (a different reading, used only to show
    that the two readings differ when cuts are truncated)."""
    Lx, Ly = lat.Lx, lat.Ly
    S = np.asarray(S)
    sig = 1 - 2 * S.astype(np.int64)
    Ud = [dense_env_down(A, lat, S, i)[0] for i in range(Ly)]
    Ld = [dense_env_up(A, lat, S, i)[0] for i in range(Ly)]
    nn, nnn = lattice_bonds(Lx, Ly)
    E = 0.0
    for bonds, J in ((nn, lat.J1), (nnn, lat.J2)):
        for m, n in bonds:
            E += J * sig[m] * sig[n] / 4.0
            if S[m] == S[n]:
                continue
            Sp = S.copy()
            Sp[m], Sp[n] = S[n], S[m]
            i = min(m, n) // Lx
            if ratio_source == "full":
                s1, l1 = dense_psi_truncated(A, lat, Sp)
                s0, l0 = dense_psi_truncated(A, lat, S)
                rho = s1 * s0 * math.exp(l1 - l0)
            elif m // Lx == n // Lx:
                rho = (dense_row_sandwich(Ud[i], A, lat, Sp, i, Ld[i]) /
                       dense_row_sandwich(Ud[i], A, lat, S, i, Ld[i]))
            else:
                rho = (dense_two_row_sandwich(Ud[i], A, lat, Sp, i, Ld[i + 1]) /
                       dense_two_row_sandwich(Ud[i], A, lat, S, i, Ld[i + 1]))
            E += J * 0.5 * rho
    return E


def mps_to_dense(mps):
    """Contract an open MPS [a, p, b] into a dense vector over its physical legs."""
    v = np.ones((1, 1))
    dims = []
    for M in mps:
        a, p, b = M.shape
        v = np.einsum("xa,apb->xpb", v, M).reshape(-1, b)
        dims.append(p)
    return v.reshape(dims)


def dense_row_sandwich(Udense, A, lat, S, i, Ldense):
    """<U| row i |L> with U, L given as dense vectors over the row's u- and d-legs."""
    out = _push_row(Udense, A, lat, S, i)
    return float(np.sum(out * Ldense))


def full_wavefunction(A, lat):
    """All amplitudes W(S) for S in {0,1}^N, index = sum_m s_m 2^(N-1-m)."""
    Lx, Ly = lat.Lx, lat.Ly
    # X[phys-so-far, boundary(d-legs of previous row / u-legs of current), h]
    X = np.ones((1, 1, 1))
    Udims = [1] * Lx
    for i in range(Ly):
        rem = list(Udims)
        X = X.reshape(X.shape[0], -1, 1)
        newd = []
        for j in range(Lx):
            dl, du, dr, dd = _dims(lat, i, j)
            Tm = A[i * Lx + j][:, :dl, :du, :dr, :dd]          # [s, l, u, r, d]
            Pphys = X.shape[0]
            done = int(np.prod(newd)) if newd else 1
            u = rem[j]
            R = int(np.prod(rem[j + 1:])) if j + 1 < Lx else 1
            H = X.shape[2]
            X5 = X.reshape(Pphys, done, u, R, H)
            Y = np.einsum("xpuRh,shurd->xspdRr", X5, Tm)
            newd.append(dd)
            X = Y.reshape(Pphys * 2, done * dd * R, dr)
        Udims = newd
    return X.reshape(-1)


def configs_from_index(N):
    idx = np.arange(2 ** N)
    return ((idx[:, None] >> (N - 1 - np.arange(N))[None, :]) & 1).astype(np.int8)


def lattice_bonds(Lx, Ly):
    nn, nnn = [], []
    for i in range(Ly):
        for j in range(Lx):
            m = i * Lx + j
            if j + 1 < Lx:
                nn.append((m, m + 1))
            if i + 1 < Ly:
                nn.append((m, m + Lx))
            if i + 1 < Ly and j + 1 < Lx:
                nnn.append((m, m + Lx + 1))
                nnn.append((m + 1, m + Lx))
    return nn, nnn


def heisenberg_j1j2(Lx, Ly, J1, J2):
    """Sparse H = J1 sum_NN S.S + J2 sum_NNN S.S on the open lattice, basis index as above."""
    N = Lx * Ly
    dim = 2 ** N
    idx = np.arange(dim, dtype=np.int64)
    diag = np.zeros(dim)
    rows, cols, vals = [], [], []
    nn, nnn = lattice_bonds(Lx, Ly)
    for bonds, J in ((nn, J1), (nnn, J2)):
        for m, n in bonds:
            bm = (idx >> (N - 1 - m)) & 1
            bn = (idx >> (N - 1 - n)) & 1
            diag += J * 0.25 * np.where(bm == bn, 1.0, -1.0)
            anti = np.nonzero(bm != bn)[0]
            flipped = anti ^ ((1 << (N - 1 - m)) | (1 << (N - 1 - n)))
            rows.append(flipped)
            cols.append(anti)
            vals.append(np.full(anti.size, 0.5 * J))
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(dim, dim))


# ---------------------------------------------------------------------------
# input transforms used by closed-form and invariance pins
# ---------------------------------------------------------------------------
def product_peps(lat, a, rng=None, junk=0.0):
    """Embed the D = 1 product state a[m][s] at bond D (entries at index 0 of every leg),
    optionally with random junk on entries no contraction may read."""
    D = lat.D
    A = np.zeros((lat.N, 2, D, D, D, D))
    A[:, :, 0, 0, 0, 0] = a
    if junk and rng is not None:
        for i in range(lat.Ly):
            for j in range(lat.Lx):
                m = i * lat.Lx + j
                dl, du, dr, dd = _dims(lat, i, j)
                mask = np.ones((D, D, D, D), dtype=bool)
                mask[:dl, :du, :dr, :dd] = False
                A[m][:, mask] = junk * rng.standard_normal((2, int(mask.sum())))
    return A


def gauge_dress(A, lat, rng, horizontal=True, vertical="orthogonal", cond=3.0):
    """Insert G G^-1 on internal bonds: horizontal bonds get random invertible G,
    vertical bonds random orthogonal (or invertible) G.  The exact network is unchanged."""
    A = A.copy()
    D = lat.D

    def rand_inv():
        M = rng.standard_normal((D, D))
        U, _, Vt = np.linalg.svd(M)
        s = np.geomspace(1.0, 1.0 / cond, D)
        return U @ np.diag(s) @ Vt

    def rand_orth():
        Qm, R = np.linalg.qr(rng.standard_normal((D, D)))
        return Qm * np.sign(np.diag(R))

    for i in range(lat.Ly):
        for j in range(lat.Lx):
            m = i * lat.Lx + j
            if horizontal and j + 1 < lat.Lx:
                G = rand_inv()
                Gi = np.linalg.inv(G)
                A[m] = np.einsum("slurd,rx->sluxd", A[m], G)
                A[m + 1] = np.einsum("xl,slurd->sxurd", Gi, A[m + 1])
            if vertical and i + 1 < lat.Ly:
                G = rand_orth() if vertical == "orthogonal" else rand_inv()
                Gi = G.T if vertical == "orthogonal" else np.linalg.inv(G)
                A[m] = np.einsum("slurd,dx->slurx", A[m], G)
                A[m + lat.Lx] = np.einsum("xu,slurd->slxrd", Gi, A[m + lat.Lx])
    return A


def spin_pair_operator(N, m, n):
    """Sparse S_m . S_n on {0,1}^N (basis index as above; s = 0 is S^z = +1/2): the
    diagonal +-1/4 and the exchange of an anti-parallel pair with element 1/2."""
    dim = 2 ** N
    idx = np.arange(dim, dtype=np.int64)
    if m == n:
        return sp.identity(dim, format="csr") * 0.75
    bm = (idx >> (N - 1 - m)) & 1
    bn = (idx >> (N - 1 - n)) & 1
    diag = 0.25 * np.where(bm == bn, 1.0, -1.0)
    anti = np.nonzero(bm != bn)[0]
    flipped = anti ^ ((1 << (N - 1 - m)) | (1 << (N - 1 - n)))
    rows = np.concatenate([idx, flipped])
    cols = np.concatenate([idx, anti])
    vals = np.concatenate([diag, np.full(anti.size, 0.5)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))
