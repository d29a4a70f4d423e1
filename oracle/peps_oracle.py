"""FP64 CPU oracle for the PEPS-VMC hot path (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  The product path (the HIP library and its Python binding) never
calls it, and it shares no code with that path.

What it computes, per spin configuration S (paper Sec. II-A):
  * W(S), the single-layer contraction of Eq. (1) at fixed S, approximated by
    the row-by-row boundary-MPS contraction with bond truncation Dc of Fig. 1(c);
  * the local energy E(S) of Eq. (4) for the J1-J2 Hamiltonian of Sec. III-A;
  * the log-derivatives Delta = B/W of Eqs. (6)-(7);
  * one Metropolis step of the sampling loop of Sec. II-B (steps 1-3): a symmetric
    exchange proposal on a J1 or J2 bond, W(S') by the same contraction, acceptance
    for the weights W(S)^2 of Eq. (3), with the uniform random numbers passed in;
  * the sampled energy (Eq. (3)) and gradient (Eq. (5)), the gradient-optimisation
    update of the tensors, and one iteration of the optimisation loop (Sec. II-B,
    Step B: sample, estimate, update), with the random step factors passed in;
  * spin-spin correlations <S_m . S_m'> (local value sigma sigma / 4 plus half the
    ratio W(S')/W(S) of the exchanged configuration, contracted in full) and the
    structure factor m_s^2(k) over a block of sites (Sec. III-A).
Everything is IEEE float64.  numpy's QR and SVD (LAPACK) are used as library
steps; contractions are written as einsum calls, one per tensor pair.

Readings of points the paper leaves open (each one is listed in the design notes):
  * boundary legs of the open lattice are restricted to index 0; other entries of
    the uniform D^4 storage are dead parameters (zero derivative);
  * truncation = canonical SVD truncation: a left-to-right QR sweep to
    left-canonical form, then a right-to-left SVD sweep keeping
    t = min(Dc, rows, cols) singular vectors (zero ones included), then the
    norm is pulled out of the first site and kept as a log;
  * the variational alternative (sweeps >= 1; Sec. II-A's O(D^4 Dc^2) cost): one-site
    alternating least squares started from the incoming boundary, used where that
    boundary already has the dims of the result, the SVD truncation elsewhere;
  * the bottom-up sweep uses the same column orientation as the top-down one;
  * the reported amplitude is the top-down one (final overlap with the last row);
  * spin-flip ratios use the sandwich that holds both sites: the single-row
    sandwich <U_i|row i|L_i> for horizontal bonds, the two-row sandwich
    <U_i|rows i,i+1|L_{i+1}> for vertical and diagonal bonds, each divided by the
    same sandwich at the unflipped S;
  * Delta_m is the frozen-environment derivative of ln|W_i| (row i holds site m);
  * s = 0 is spin up (S^z = +1/2), sigma = 1 - 2s; S_i.S_j = sigma_i sigma_j / 4
    plus 1/2 for the exchange of an anti-parallel pair (no sign rotation);
  * the Metropolis proposal (the paper names none): exchange the spins of a bond drawn
    uniformly from every J1 and J2 bond (it conserves S^z and undoes itself); a bond of
    equal spins is no move; W(S') comes from a full contraction of S', as in the
    paper's step 2.

Parity pins live in the test suite: dense transfer-matrix contraction (exact
regime), dense sequential Schmidt projection (truncated regime), brute force
over all 2^16 configurations of a 4x4 lattice, closed forms of product states,
finite differences and invariants.
"""
from __future__ import annotations

import math

import numpy as np

# Per-sample status flags (same meaning as the library's).
FLAG_OK, FLAG_BAD_CONFIG, FLAG_ZERO_AMPLITUDE, FLAG_NONFINITE = 0, 1, 2, 3


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def leg_dims(lat, i, j):
    """(Dl, Du, Dr, Dd) of site (i, j): outward legs of the open lattice have dim 1."""
    D = lat.D
    return (1 if j == 0 else D, 1 if i == 0 else D,
            1 if j == lat.Lx - 1 else D, 1 if i == lat.Ly - 1 else D)


def site_tensor(A, lat, i, j, s):
    """T = A_m^{s} of Eq. (1) as a rank-4 tensor [l, u, r, d] (m = i*Lx + j)."""
    Dl, Du, Dr, Dd = leg_dims(lat, i, j)
    return A[i * lat.Lx + j, s, :Dl, :Du, :Dr, :Dd]


def row_tensors(A, lat, S, i):
    return [site_tensor(A, lat, i, j, int(S[i * lat.Lx + j])) for j in range(lat.Lx)]


def j1_bonds(lat):
    """Nearest-neighbour pairs <i,j> of the open lattice (Sec. III-A): (site, site, kind)."""
    out = []
    for i in range(lat.Ly):
        for j in range(lat.Lx):
            m = i * lat.Lx + j
            if j + 1 < lat.Lx:
                out.append((m, m + 1, "h"))
            if i + 1 < lat.Ly:
                out.append((m, m + lat.Lx, "v"))
    return out


def j2_bonds(lat):
    """Next-nearest-neighbour pairs <<i,j>>: both diagonals of every plaquette."""
    out = []
    for i in range(lat.Ly - 1):
        for j in range(lat.Lx - 1):
            m = i * lat.Lx + j
            out.append((m, m + lat.Lx + 1, "d"))      # (i,j)-(i+1,j+1)
            out.append((m + 1, m + lat.Lx, "a"))      # (i,j+1)-(i+1,j)
    return out


def _c(spec, x, y):
    """One pairwise contraction (a tensordot), the only contraction primitive used here."""
    return np.einsum(spec, x, y, optimize=True)


def _row_step(P, Uj, T, Lj):
    """P_{j+1}[b,r,c] = sum_{a,l,e,u,d} P_j[a,l,e] U_j[a,u,b] T_j[l,u,r,d] L_j[e,d,c]."""
    Y = _c("ale,aub->leub", P, Uj)
    Y = _c("leub,lurd->ebrd", Y, T)
    return _c("ebrd,edc->brc", Y, Lj)


def _row_step_right(Uj, T, Lj, Q):
    """Q_j[a,l,e] = sum U_j[a,u,b] T_j[l,u,r,d] L_j[e,d,c] Q_{j+1}[b,r,c]."""
    Y = _c("edc,brc->edbr", Lj, Q)
    Y = _c("lurd,edbr->lueb", T, Y)
    return _c("aub,lueb->ale", Uj, Y)


def _two_row_step(P, Uj, T1, T2, Lj):
    """P_{j+1}[b,r,s,c] = sum P_j[a,x,y,e] U_j[a,u,b] T1[x,u,r,m] T2[y,m,s,q] L_j[e,q,c]."""
    Y = _c("axye,aub->xyeub", P, Uj)
    Y = _c("xyeub,xurm->yebrm", Y, T1)
    Y = _c("yebrm,ymsq->ebrsq", Y, T2)
    return _c("ebrsq,eqc->brsc", Y, Lj)


def _rescale(x):
    """x / c and ln c with c = max|x| (c = 1 if x is all zero): keeps partials in range."""
    c = float(np.max(np.abs(x))) if x.size else 0.0
    if c == 0.0 or not math.isfinite(c):
        return x, 0.0
    return x / c, math.log(c)


# --------------------------------------------------------------------------
# boundary MPS: apply a row, truncate to Dc (Fig. 1(c))
# --------------------------------------------------------------------------
def trivial_mps(Lx):
    """Boundary MPS of bond 1 and physical dim 1 (index 0 on the outward legs)."""
    return [np.ones((1, 1, 1)) for _ in range(Lx)]


def apply_row_down(U, row):
    """Exact product of row i (as an MPO acting on its u-legs) with the MPS U_i.
    C_j[(a,l), d, (b,r)] = sum_u U_j[a,u,b] T_j[l,u,r,d]: bond chi*D, physical d."""
    out = []
    for Uj, T in zip(U, row):
        a, _, b = Uj.shape
        l, _, r, d = T.shape
        out.append(np.einsum("aub,lurd->aldbr", Uj, T).reshape(a * l, d, b * r))
    return out


def apply_row_up(L, row):
    """Mirror of apply_row_down for the bottom-up sweep: contract the d-legs, keep u."""
    out = []
    for Lj, T in zip(L, row):
        a, _, b = Lj.shape
        l, u, r, _ = T.shape
        out.append(np.einsum("adb,lurd->alubr", Lj, T).reshape(a * l, u, b * r))
    return out


def truncate(mps, Dc):
    """Canonical truncation of an open MPS to bond <= Dc.

    Left-to-right QR sweep (left-canonical form), then right-to-left SVD sweep
    keeping the t = min(Dc, rows, cols) largest singular values at every cut,
    then the norm nu of the first site is pulled out.  Returns (mps, ln nu);
    ln nu = -inf for the zero state.
    """
    mps = [x.copy() for x in mps]
    n = len(mps)
    for j in range(n - 1):
        a, p, b = mps[j].shape
        Q, R = np.linalg.qr(mps[j].reshape(a * p, b), mode="reduced")
        mps[j] = Q.reshape(a, p, Q.shape[1])
        mps[j + 1] = np.einsum("kb,bpc->kpc", R, mps[j + 1])
    for j in range(n - 1, 0, -1):
        a, p, b = mps[j].shape
        Um, sv, Vt = np.linalg.svd(mps[j].reshape(a, p * b), full_matrices=False)
        t = min(Dc, a, p * b)
        mps[j] = Vt[:t].reshape(t, p, b)
        mps[j - 1] = np.einsum("apk,kt->apt", mps[j - 1], Um[:, :t] * sv[:t])
    nu = float(np.linalg.norm(mps[0]))
    if nu == 0.0:
        return mps, -math.inf
    mps[0] = mps[0] / nu
    return mps, math.log(nu)


# --------------------------------------------------------------------------
# variational boundary compression (the GEMM-dominated alternative to the SVD
# truncation; cost O(D^4 Dc^2) per site and sweep, Sec. II-A)
# --------------------------------------------------------------------------
def truncated_bonds(mps, Dc):
    """Bond dims [1, t_1, ..., t_{n-1}, 1] that truncate(mps, Dc) produces, from the
    shapes alone: the QR sweep leaves r_{j+1} = min(r_j p_j, b_{j+1}), the SVD sweep
    keeps t_j = min(Dc, r_j, p_j t_{j+1})."""
    n = len(mps)
    r = [1] * (n + 1)
    for j in range(n - 1):
        _, p, b = mps[j].shape
        r[j + 1] = min(r[j] * p, b)
    t = [1] * (n + 1)
    for j in range(n - 1, 0, -1):
        t[j] = min(Dc, r[j], mps[j].shape[1] * t[j + 1])
    return t


def _qr_pos(M):
    """Thin QR of a tall matrix with the diagonal of R made non-negative, so that Q is
    unique when M has full column rank (numpy's LAPACK QR as the library step)."""
    Q, R = np.linalg.qr(M, mode="reduced")
    s = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * s, R * s[:, None]


def compress_variational(P, G, sweeps):
    """Variational compression of the MPS P onto the bond dims of the guess G.

    The approximation C minimises ||P - C|| one tensor at a time (one-site
    alternating least squares).  With every other tensor of C an isometry towards
    the site being updated, the optimal tensor is the contraction of P with the rest
    of C: M_j[c,d,c'] = sum L_j[c,k] P_j[k,d,k'] R_{j+1}[c',k'], where L_j (R_{j+1})
    is the overlap of C's and P's sites left of j (right of j).  Steps:
      1. bring G to right-canonical form: from the last site down to site 1, an LQ
         factorisation of each tensor (as a matrix bond x (phys bond)) keeps the
         orthonormal rows and pushes the triangular factor into the left neighbour;
      2. a sweep: sites 0..n-2 left to right (update, thin QR, keep Q, extend L),
         then sites n-1..1 right to left (update, LQ, keep the rows, extend R),
         then the update of site 0, which carries the norm;
      3. after the last sweep the norm nu of site 0 is pulled out.
    Every QR/LQ factor is sign-fixed (non-negative diagonal).  Returns (C, ln nu);
    ln nu = -inf for the zero state.
    """
    if sweeps < 1:
        raise ValueError("at least one sweep")
    n = len(P)
    C = [g.copy() for g in G]
    for j in range(n - 1, 0, -1):
        a, p, b = C[j].shape
        Q, R = _qr_pos(C[j].reshape(a, p * b).T)          # C_j = R^T Q^T
        C[j] = Q.T.reshape(a, p, b)
        C[j - 1] = _c("xpa,ka->xpk", C[j - 1], R)

    def update(j):
        X = _c("kdf,ef->kde", P[j], Renv[j + 1])            # contract P's right bond
        return _c("ck,kde->cde", Lenv[j], X)

    def left_step(j):
        X = _c("ck,cde->kde", Lenv[j], C[j])
        return _c("kde,kdf->ef", X, P[j])

    def right_step(j):
        X = _c("cde,ef->cdf", C[j], Renv[j + 1])
        return _c("cdf,kdf->ck", X, P[j])

    Lenv = [None] * (n + 1)
    Renv = [None] * (n + 1)
    Lenv[0] = np.ones((1, 1))
    Renv[n] = np.ones((1, 1))
    for j in range(n - 1, 0, -1):
        Renv[j] = right_step(j)
    for _ in range(sweeps):
        for j in range(n - 1):
            M = update(j)
            a, p, b = M.shape
            Q, _ = _qr_pos(M.reshape(a * p, b))
            C[j] = Q.reshape(a, p, b)
            Lenv[j + 1] = left_step(j)
        for j in range(n - 1, 0, -1):
            M = update(j)
            a, p, b = M.shape
            Q, _ = _qr_pos(M.reshape(a, p * b).T)
            C[j] = Q.T.reshape(a, p, b)
            Renv[j] = right_step(j)
        C[0] = update(0)
    nu = float(np.linalg.norm(C[0]))
    if nu == 0.0:
        return C, -math.inf
    C[0] = C[0] / nu
    return C, math.log(nu)


def next_boundary(E, P, Dc, sweeps=0):
    """The truncated boundary Trunc(P) of the applied MPS P = Apply(E, row).

    sweeps = 0: canonical SVD truncation.  sweeps >= 1: variational compression with
    the incoming boundary E as the guess, wherever E already has the bond and
    physical dims of the result (the bond has stopped growing); elsewhere the SVD
    truncation, which then also fixes those dims.
    """
    if sweeps > 0:
        t = truncated_bonds(P, Dc)
        if ([e.shape[0] for e in E] + [1] == t
                and all(e.shape[1] == q.shape[1] for e, q in zip(E, P))):
            return compress_variational(P, E, sweeps)
    return truncate(P, Dc)


def boundary_envs(A, lat, S, sweeps=0):
    """Upper envs U_0..U_{Ly-1} and lower envs L_0..L_{Ly-1} with their log scales.

    U_0 and L_{Ly-1} are trivial; U_{i+1} = Trunc(Apply(U_i, row i)) and
    L_{i-1} = Trunc(Apply_up(L_i, row i)), Trunc as in next_boundary.  True env =
    exp(log) * stored MPS.
    """
    Ly = lat.Ly
    U = [None] * Ly
    L = [None] * Ly
    logU = [0.0] * Ly
    logL = [0.0] * Ly
    U[0] = trivial_mps(lat.Lx)
    for i in range(Ly - 1):
        U[i + 1], ln = next_boundary(U[i], apply_row_down(U[i], row_tensors(A, lat, S, i)), lat.Dc, sweeps)
        logU[i + 1] = logU[i] + ln
    L[Ly - 1] = trivial_mps(lat.Lx)
    for i in range(Ly - 1, 0, -1):
        L[i - 1], ln = next_boundary(L[i], apply_row_up(L[i], row_tensors(A, lat, S, i)), lat.Dc, sweeps)
        logL[i - 1] = logL[i] + ln
    return U, L, logU, logL


def final_overlap(Ulast, row_last):
    """w = <U_{Ly-1}| last row> with the last row's d-legs at index 0."""
    v = np.ones((1, 1))
    for Uj, T in zip(Ulast, row_last):
        v = np.einsum("al,aub,lur->br", v, Uj, T[:, :, :, 0])
    return float(v[0, 0])


# --------------------------------------------------------------------------
# sandwiches <U_i| row(s) |L>
# --------------------------------------------------------------------------
def row_sandwich(Ui, row, Li):
    """(sign, ln|.|) of <U_i| row i |L_i> contracted column by column (no truncation)."""
    P = np.ones((1, 1, 1))
    logs = 0.0
    for Uj, T, Lj in zip(Ui, row, Li):
        P, ln = _rescale(_row_step(P, Uj, T, Lj))
        logs += ln
    w = float(P[0, 0, 0])
    return (0, -math.inf) if w == 0.0 else (int(np.sign(w)), logs + math.log(abs(w)))


def two_row_sandwich(Ui, row1, row2, Lk):
    """(sign, ln|.|) of <U_i| row i, row i+1 |L_{i+1}>."""
    P = np.ones((1, 1, 1, 1))
    logs = 0.0
    for Uj, T1, T2, Lj in zip(Ui, row1, row2, Lk):
        P, ln = _rescale(_two_row_step(P, Uj, T1, T2, Lj))
        logs += ln
    w = float(P[0, 0, 0, 0])
    return (0, -math.inf) if w == 0.0 else (int(np.sign(w)), logs + math.log(abs(w)))


def _ratio(num, den):
    """W(S')/W(S) from two (sign, log) pairs."""
    if num[0] == 0:
        return 0.0
    return num[0] * den[0] * math.exp(num[1] - den[1])


# --------------------------------------------------------------------------
# per-sample results
# --------------------------------------------------------------------------
def _check_config(lat, S):
    S = np.asarray(S)
    return S.shape == (lat.N,) and bool(np.all((S == 0) | (S == 1)))


def log_amplitude_one(A, lat, S, sweeps=0):
    """(ln|W(S)|, sign W(S), flag) from the top-down boundary-MPS contraction
    (sweeps: the truncation of next_boundary)."""
    if not _check_config(lat, S):
        return math.nan, 0, FLAG_BAD_CONFIG
    U = trivial_mps(lat.Lx)
    logscale = 0.0
    for i in range(lat.Ly - 1):
        U, ln = next_boundary(U, apply_row_down(U, row_tensors(A, lat, S, i)), lat.Dc, sweeps)
        logscale += ln
    w = final_overlap(U, row_tensors(A, lat, S, lat.Ly - 1))
    if w == 0.0 or not math.isfinite(logscale):
        return -math.inf, 0, FLAG_ZERO_AMPLITUDE
    out = logscale + math.log(abs(w))
    if not math.isfinite(out):
        return out, int(np.sign(w)), FLAG_NONFINITE
    return out, int(np.sign(w)), FLAG_OK


def local_energy_one(A, lat, S, envs=None, sweeps=0):
    """E(S) of Eq. (4) for H = J1 sum_<ij> S_i.S_j + J2 sum_<<ij>> S_i.S_j.

    Off-diagonal terms: 1/2 * W(S')/W(S) for every anti-parallel bond, where S'
    exchanges the two spins; W(S')/W(S) is taken from the sandwich that holds
    both sites, with the cached upper and lower environments.
    """
    S = np.asarray(S)
    if not _check_config(lat, S):
        return math.nan
    U, L, _, _ = envs if envs is not None else boundary_envs(A, lat, S, sweeps)
    sig = 1 - 2 * S.astype(np.int64)
    Lx = lat.Lx

    row_den = {}
    pair_den = {}

    def w_row(i, Sx):
        return row_sandwich(U[i], row_tensors(A, lat, Sx, i), L[i])

    def w_pair(i, Sx):
        return two_row_sandwich(U[i], row_tensors(A, lat, Sx, i),
                                row_tensors(A, lat, Sx, i + 1), L[i + 1])

    E = 0.0
    for bonds, J in ((j1_bonds(lat), lat.J1), (j2_bonds(lat), lat.J2)):
        for m, n, kind in bonds:
            E += J * sig[m] * sig[n] / 4.0
            if S[m] == S[n]:
                continue
            Sp = S.copy()
            Sp[m], Sp[n] = S[n], S[m]
            i = min(m, n) // Lx
            if kind == "h":
                if i not in row_den:
                    row_den[i] = w_row(i, S)
                rho = _ratio(w_row(i, Sp), row_den[i])
            else:
                if i not in pair_den:
                    pair_den[i] = w_pair(i, S)
                rho = _ratio(w_pair(i, Sp), pair_den[i])
            E += J * 0.5 * rho
    return E


def log_derivative_one(A, lat, S, envs=None, sweeps=0):
    """Delta[m][s][l][u][r][d] = (1/W_i) dW_i/dA_m^{s}, Eqs. (6)-(7), frozen environments.

    B_m is the row-i sandwich with site m removed: left partial P_j (columns < j),
    the environment legs U_i[j], L_i[j], and right partial Q_{j+1} (columns > j).
    Only the slice s = S[m] and the live (non-outward) leg entries are non-zero.
    """
    S = np.asarray(S)
    D, Lx, Ly = lat.D, lat.Lx, lat.Ly
    out = np.zeros((lat.N, 2, D, D, D, D))
    if not _check_config(lat, S):
        out[:] = np.nan
        return out
    U, L, _, _ = envs if envs is not None else boundary_envs(A, lat, S, sweeps)
    for i in range(Ly):
        row = row_tensors(A, lat, S, i)
        left = [(np.ones((1, 1, 1)), 0.0)]
        for j in range(Lx):
            P, lg = left[-1]
            P, ln = _rescale(_row_step(P, U[i][j], row[j], L[i][j]))
            left.append((P, lg + ln))
        right = [None] * (Lx + 1)
        right[Lx] = (np.ones((1, 1, 1)), 0.0)
        for j in range(Lx - 1, -1, -1):
            Q, lg = right[j + 1]
            Q, ln = _rescale(_row_step_right(U[i][j], row[j], L[i][j], Q))
            right[j] = (Q, lg + ln)
        Pn, lgn = left[Lx]
        w = float(Pn[0, 0, 0])
        if w == 0.0:
            continue
        for j in range(Lx):
            P, lp = left[j]
            Q, lq = right[j + 1]
            B = _c("leub,edbr->lurd", _c("ale,aub->leub", P, U[i][j]),
                   _c("edc,brc->edbr", L[i][j], Q))
            m = i * Lx + j
            Dl, Du, Dr, Dd = leg_dims(lat, i, j)
            out[m, int(S[m]), :Dl, :Du, :Dr, :Dd] = B / w * math.exp(lp + lq - lgn)
    return out


# --------------------------------------------------------------------------
# batched front ends (plain loops over samples)
# --------------------------------------------------------------------------
def log_amplitude(A, lat, S, sweeps=0):
    B = S.shape[0]
    la = np.empty(B)
    sg = np.empty(B, dtype=np.int8)
    fl = np.empty(B, dtype=np.int8)
    for b in range(B):
        la[b], sg[b], fl[b] = log_amplitude_one(A, lat, S[b], sweeps)
    return la, sg, fl


def local_energy(A, lat, S, sweeps=0):
    """(log_abs, sign, e_loc, flags) per sample."""
    B = S.shape[0]
    la, sg, fl = log_amplitude(A, lat, S, sweeps)
    e = np.full(B, np.nan)
    for b in range(B):
        if fl[b] == FLAG_OK:
            e[b] = local_energy_one(A, lat, S[b], sweeps=sweeps)
            if not math.isfinite(e[b]):
                fl[b] = FLAG_NONFINITE
    return la, sg, e, fl


def log_derivative(A, lat, S, weights=None, sweeps=0):
    """Per-sample Delta [B][N][2][D^4] or, with weights, sum_b weights[b] * Delta_b
    accumulated in sample order (the per-sample term of Eq. (5))."""
    B = S.shape[0]
    D4 = lat.D ** 4
    if weights is None:
        out = np.zeros((B, lat.N, 2, D4))
        for b in range(B):
            out[b] = log_derivative_one(A, lat, S[b], sweeps=sweeps).reshape(lat.N, 2, D4)
        return out
    g = np.zeros((lat.N, 2, D4))
    for b in range(B):
        g += weights[b] * log_derivative_one(A, lat, S[b], sweeps=sweeps).reshape(lat.N, 2, D4)
    return g


def full_path_one(A, lat, S, sweeps=0):
    """Amplitude, local energy and log-derivative of one sample from one set of envs."""
    la, sg, fl = log_amplitude_one(A, lat, S, sweeps)
    if fl != FLAG_OK:
        return la, sg, math.nan, np.zeros((lat.N, 2, lat.D ** 4)), fl
    envs = boundary_envs(A, lat, S, sweeps)
    e = local_energy_one(A, lat, S, envs)
    d = log_derivative_one(A, lat, S, envs).reshape(lat.N, 2, -1)
    return la, sg, e, d, fl


# --------------------------------------------------------------------------
# Metropolis sampling (Sec. II-B, steps 1-3 of the sampling loop; weights W(S)^2 of
# the energy estimator, Eq. (3))
# --------------------------------------------------------------------------
def proposal_bonds(lat):
    """The exchange moves a Metropolis step draws from, in a fixed order: horizontal
    pairs (i,j)-(i,j+1) row by row, then vertical (i,j)-(i+1,j), then the diagonals
    (i,j)-(i+1,j+1), then the anti-diagonals (i,j+1)-(i+1,j): every J1 and J2 bond once."""
    Lx, Ly = lat.Lx, lat.Ly
    out = [(i * Lx + j, i * Lx + j + 1) for i in range(Ly) for j in range(Lx - 1)]
    out += [(i * Lx + j, (i + 1) * Lx + j) for i in range(Ly - 1) for j in range(Lx)]
    out += [(i * Lx + j, (i + 1) * Lx + j + 1) for i in range(Ly - 1) for j in range(Lx - 1)]
    out += [(i * Lx + j + 1, (i + 1) * Lx + j) for i in range(Ly - 1) for j in range(Lx - 1)]
    return out


def metropolis_step(A, lat, S, u, log_abs, sign, sweeps=0):
    """One Metropolis step of every chain.  Chain b proposes the exchange of the two
    spins of bond k = min(floor(u[b,0] nb), nb - 1) of proposal_bonds (a symmetric
    proposal: the same bond undoes it; a pair of equal spins is no move), contracts
    W(S') like log_amplitude, and moves to S' when u[b,1] < W(S')^2 / W(S)^2 (the
    Metropolis rule for weights W^2) and S' has flag 0.
    log_abs, sign: ln|W(S)| and sign of the current configurations; sweeps: the
    truncation of next_boundary.  Returns (S, log_abs, sign, accepted), new arrays."""
    bonds = proposal_bonds(lat)
    nb = len(bonds)
    S = np.array(S, dtype=np.int8, copy=True)
    la = np.array(log_abs, dtype=np.float64, copy=True)
    sg = np.array(sign, dtype=np.int8, copy=True)
    acc = np.zeros(S.shape[0], dtype=np.int8)
    for b in range(S.shape[0]):
        m, n = bonds[min(int(u[b, 0] * nb), nb - 1)]
        if S[b, m] == S[b, n]:
            continue
        Sp = S[b].copy()
        Sp[m], Sp[n] = S[b, n], S[b, m]
        lap, sgp, flp = log_amplitude_one(A, lat, Sp, sweeps)
        if flp != FLAG_OK:
            continue
        if u[b, 1] < math.exp(min(2.0 * (lap - la[b]), 700.0)):
            S[b], la[b], sg[b], acc[b] = Sp, lap, sgp, 1
    return S, la, sg, acc


# --------------------------------------------------------------------------
# Monte Carlo estimators and the gradient-optimisation step (Sec. II-A: the sampled
# energy of Eq. (3), its gradient Eq. (5), the GO update of the tensors; Sec. II-B:
# one iteration of the GO main loop, Step B)
# --------------------------------------------------------------------------
def energy_gradient(A, lat, S, weights=None):
    """Monte Carlo energy and energy gradient over the samples with flag 0.
    <x> is the sample mean (weights None: every sample counts once; else the weighted
    mean sum_b w_b x_b / sum_b w_b).  E = <E(S)> (the sampled form of Eq. (3)) and
    dE/dA = 2 <Delta E> - 2 <Delta> <E> (Eq. (5)).
    Returns (E, count, grad [N][2][D^4], e_loc, flags)."""
    _, _, e, fl = local_energy(A, lat, S)
    ok = fl == FLAG_OK
    w = np.ones(S.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64)
    w = np.where(ok, w, 0.0)
    tot = w.sum()
    count = int(ok.sum())
    if count == 0 or tot == 0.0:
        return math.nan, count, np.zeros((lat.N, 2, lat.D ** 4)), e, fl
    Em = float((w[ok] * e[ok]).sum() / tot)
    dE = np.zeros((lat.N, 2, lat.D ** 4))
    dm = np.zeros_like(dE)
    for b in np.nonzero(ok)[0]:
        d = log_derivative_one(A, lat, S[b]).reshape(lat.N, 2, -1)
        dE += (w[b] / tot) * e[b] * d
        dm += (w[b] / tot) * d
    return Em, count, 2.0 * dE - 2.0 * dm * Em, e, fl


def go_update(A, grad, p, dt):
    """Gradient-optimisation rule: every element moves against the sign of its energy
    derivative by p * dt(n), p in (0, 1) drawn per element (passed in).  A zero (or NaN)
    derivative leaves the element where it is.  Returns a new array."""
    g = np.asarray(grad, dtype=np.float64).reshape(np.shape(A))
    s = np.where(g > 0, 1.0, np.where(g < 0, -1.0, 0.0))
    step = np.asarray(p, dtype=np.float64).reshape(np.shape(A)) * dt
    return np.asarray(A, dtype=np.float64) - step * s


def vmc_step(A, lat, S, u, p, dt):
    """One iteration of the GO main loop: ln|W| of the chains S under A, len(u)
    Metropolis steps of every chain (u[t] are the uniforms of step t), the energy and
    gradient over the chains' configurations, then the GO update with the per-element
    p and the step dt.  Returns (A_new, S, E, count, grad)."""
    la, sg, _ = log_amplitude(A, lat, S)
    for t in range(len(u)):
        S, la, sg, _ = metropolis_step(A, lat, S, u[t], la, sg)
    E, count, grad, _, _ = energy_gradient(A, lat, S)
    return go_update(A, grad, p, dt), S, E, count, grad


# --------------------------------------------------------------------------
# Spin-spin correlations (Sec. III-A: <S_m . S_m'> and the structure factor m_s^2(k))
# --------------------------------------------------------------------------
def pair_correlation_one(A, lat, S, m, n, la=None, sg=None, sweeps=0):
    """Local value of S_m . S_n at configuration S: sigma_m sigma_n / 4, plus 1/2 W(S')/W(S)
    when the two spins differ (S' = S with them exchanged), W(S') from a full contraction;
    3/4 when m == n.  Returns (value, flag): the flag of S, or FLAG_NONFINITE when the
    contraction of S' is not finite (a zero W(S') just gives a zero ratio)."""
    if la is None:
        la, sg, fl = log_amplitude_one(A, lat, S, sweeps)
        if fl != FLAG_OK:
            return math.nan, fl
    if m == n:
        return 0.75, FLAG_OK
    sm, sn = 1 - 2 * int(S[m]), 1 - 2 * int(S[n])
    v = 0.25 * sm * sn
    if S[m] != S[n]:
        Sp = np.array(S, dtype=np.int8, copy=True)
        Sp[m], Sp[n] = S[n], S[m]
        lap, sgp, flp = log_amplitude_one(A, lat, Sp, sweeps)
        if flp == FLAG_ZERO_AMPLITUDE:
            return v, FLAG_OK
        if flp != FLAG_OK:
            return math.nan, FLAG_NONFINITE
        v += 0.5 * sgp * sg * math.exp(lap - la)
    return v, FLAG_OK


def pair_correlations(A, lat, S, pairs, weights=None, sweeps=0):
    """Monte Carlo mean of S_m . S_n for every (m, n) in pairs over the samples whose
    configuration and exchanged configurations all contract (flag 0); weights as in
    energy_gradient.  Returns (means [P], per-sample values [B][P], flags [B])."""
    B, P = S.shape[0], len(pairs)
    vals = np.full((B, P), np.nan)
    fl = np.zeros(B, dtype=np.int8)
    for b in range(B):
        la, sg, f = log_amplitude_one(A, lat, S[b], sweeps)
        if f != FLAG_OK:
            fl[b] = f
            continue
        for k, (m, n) in enumerate(pairs):
            vals[b, k], f = pair_correlation_one(A, lat, S[b], m, n, la, sg, sweeps)
            if f != FLAG_OK:
                fl[b] = f
                break
    ok = fl == FLAG_OK
    w = np.ones(B) if weights is None else np.asarray(weights, dtype=np.float64)
    w = np.where(ok, w, 0.0)
    if w.sum() == 0.0:
        return np.full(P, np.nan), vals, fl
    means = (w[ok, None] * vals[ok]).sum(0) / w.sum()
    return means, vals, fl


def structure_factor(lat, sites, corr, ks):
    """m_s^2(k) = (1 / Nb^2) sum_{m, m' in sites} <S_m . S_m'> exp(i k . (r_m - r_m'))
    for each k = (kx, ky), with r_m = (column, row) of site m and Nb = len(sites).
    corr: the full matrix <S_m . S_m'> over `sites` (diagonal 3/4).  Returns real parts."""
    r = np.array([(s % lat.Lx, s // lat.Lx) for s in sites], dtype=np.float64)
    out = []
    for kx, ky in ks:
        ph = np.exp(1j * (kx * r[:, 0] + ky * r[:, 1]))
        out.append(float(np.real(ph @ corr @ np.conj(ph))) / len(sites) ** 2)
    return np.array(out)


def bulk_sites(lat, margin=2):
    """Sites of the central (Lx - 2 margin) x (Ly - 2 margin) block, row-major."""
    return [i * lat.Lx + j for i in range(margin, lat.Ly - margin) for j in range(margin, lat.Lx - margin)]
