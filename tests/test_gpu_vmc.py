"""Optimisation-loop step on the GPU (peps_go_update, peps_vmc_step, through the C ABI)
against the FP64 oracle.

The GO update is elementwise with exactly rounded arithmetic on both sides, so it is
compared bit for bit.  In a whole step the sign of each gradient element decides the
move; where the oracle's gradient element is within the gradient tolerance of zero both
signs are valid, and there the test only checks that the element moved by 0 or p*dt.
"""
import sys

import numpy as np
import pytest

import oracle as O
import pins_lib as P
from paper_1806_03761_amd.workloads import Lattice, make_random, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _peps():
    from paper_1806_03761_amd import peps
    return peps


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("shape", [(64, 2, 4, 4, 4, 4), (15, 2, 3, 3, 3, 3)])
def test_go_update_bitwise(shape):
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal(shape)
    g = rng.standard_normal(shape)
    g.reshape(-1)[::7] = 0.0
    g.reshape(-1)[3::97] = np.nan
    p = rng.uniform(0.0, 1.0, shape)
    lat = Lattice(8, 8, 4, 16) if shape[0] == 64 else Lattice(3, 5, 3, 5)
    _say("GO update", shape)
    Ad = _cuda(A)
    _peps().go_update(Ad, _cuda(g), _cuda(p), lat, 0.0125)
    torch.cuda.synchronize()
    want = O.go_update(A, g, p, 0.0125)
    assert np.array_equal(Ad.cpu().numpy(), want)


def _check_step(A0, A_g, S_g, E_g, g_g, lat, S0, u, p, dt, tol_g, tol_e):
    A_o, S_o, E_o, cnt_o, g_o = O.vmc_step(A0, lat, S0, u, p, dt)
    g_o, g_g = g_o.reshape(A0.shape), g_g.reshape(A0.shape)
    assert np.array_equal(S_g, S_o)
    assert E_g[1] == cnt_o
    assert abs(E_g[0] - E_o) <= tol_e * max(1.0, abs(E_o)), (E_g[0], E_o)
    assert np.linalg.norm(g_g - g_o) <= tol_g * np.linalg.norm(g_o)
    # elements whose derivative sign is unambiguous move exactly as the oracle's
    sure = np.abs(g_o) > 10 * tol_g * np.abs(g_o).max()
    assert np.array_equal(A_g[sure], A_o[sure])
    moved = np.abs(A_g - A0)
    step = (p * dt).reshape(A0.shape)
    ulp = 4 * np.finfo(np.float64).eps * np.abs(A0).max()
    assert np.all((moved == 0.0) | (np.abs(moved - step) <= ulp))
    return A_o, S_o


def test_vmc_step_4x4_matches_oracle():
    """4x4 D2 Dc4, 64 chains, two loop iterations of 3 Metropolis steps each, f64."""
    peps = _peps()
    lat, A, S, _ = make_workload("4x4_D2_Dc4", 64)
    rng = np.random.default_rng(21)
    Ad, Sd = _cuda(A), _cuda(S)
    for it in range(2):
        u = rng.random((3, S.shape[0], 2))
        p = rng.uniform(0.0, 1.0, A.shape)
        _say("4x4 VMC step", it)
        E, g = peps.vmc_step(Ad, Sd, lat, _cuda(u), _cuda(p), 0.01, "f64")
        torch.cuda.synchronize()
        A_g, S_g = Ad.cpu().numpy(), Sd.cpu().numpy()
        A_o, S_o = _check_step(A, A_g, S_g, E.cpu().numpy(), g.cpu().numpy(), lat, S, u, p, 0.01,
                               1e-9, 1e-10)
        # a second iteration only from tensors the two sides agree on bit for bit
        if not np.array_equal(A_o, A_g):
            break
        A, S = A_o, S_o


def test_vmc_step_ragged_no_sampling():
    """3x5 D3 Dc5, 37 chains, n_mc = 0 (estimate and update only); the same step with
    the gradient kept inside the library moves A identically; batch 0 is an error."""
    peps = _peps()
    lat = Lattice(3, 5, 3, 5)
    A, S = make_random(lat, 37, 91)
    rng = np.random.default_rng(4)
    p = rng.uniform(0.0, 1.0, A.shape)
    Ad, Sd = _cuda(A), _cuda(S)
    _say("3x5 VMC step, n_mc 0")
    u = torch.zeros((0, S.shape[0], 2), dtype=torch.float64, device="cuda")
    E, g = peps.vmc_step(Ad, Sd, lat, u, _cuda(p), 0.003, "f64")
    torch.cuda.synchronize()
    _check_step(A, Ad.cpu().numpy(), Sd.cpu().numpy(), E.cpu().numpy(), g.cpu().numpy(), lat, S,
                np.zeros((0, S.shape[0], 2)), p, 0.003, 1e-9, 1e-10)
    A2 = _cuda(A)
    E2, g2 = peps.vmc_step(A2, _cuda(S), lat, u, _cuda(p), 0.003, "f64", return_grad=False)
    assert g2 is None and torch.equal(A2, Ad) and torch.equal(E2, E)
    with pytest.raises(peps.PepsError):
        peps.vmc_step(Ad, Sd[:0], lat, u[:, :0], _cuda(p), 0.003, "f64")


@pytest.mark.parametrize("prec", ["f32"])
def test_vmc_step_8x8_full_batch_is_its_parts(prec):
    """8x8 D4 Dc16 with 4096 chains (the benchmark's batch): one loop iteration equals,
    bit for bit, the entry points it is made of run one after another (each of them
    checked against the oracle in the other tests); the sampled energy is the mean
    local energy of the final chains."""
    peps = _peps()
    lat, A, S, _ = make_workload("8x8_D4_Dc16")
    rng = np.random.default_rng(8)
    u = _cuda(rng.random((2, S.shape[0], 2)))
    p = _cuda(rng.uniform(0.0, 1.0, A.shape))
    _say("8x8 VMC step, 4096 chains", prec)
    A1, S1 = _cuda(A), _cuda(S)
    E1, g1 = peps.vmc_step(A1, S1, lat, u, p, 0.002, prec)
    A2, S2 = _cuda(A), _cuda(S)
    la, sg, _ = peps.log_amplitude(A2, S2, lat, prec)
    for t in range(2):
        peps.metropolis_step(A2, S2, lat, u[t], la, sg, prec)
    _, _, e, g2, fl = peps.evaluate(A2, S2, lat, prec, grad_mode=3)
    peps.go_update(A2, g2, p, lat, 0.002)
    torch.cuda.synchronize()
    assert torch.equal(S1, S2)
    assert torch.equal(g1.reshape(g2.shape), g2)
    assert torch.equal(A1, A2)
    ok = fl == 0
    E1 = E1.cpu().numpy()
    assert E1[1] == int(ok.sum().item())
    Em = e[ok].double().mean().item()
    assert abs(E1[0] - Em) <= 1e-12 * abs(Em)


def test_vmc_lowers_the_exact_energy_4x2():
    """Exact regime (4x2, D2, Dc4), 1024 chains: four loop iterations (8 Metropolis
    steps, dt = 0.02) lower the exact energy of the S^z = 0 sector (dense contraction and
    sparse Hamiltonian on the CPU) at every iteration."""
    peps = _peps()
    lat = Lattice(4, 2, 2, 4)
    A, S = make_random(lat, 1024, 45)
    cfg = P.configs_from_index(lat.N)
    cfg = cfg[cfg.sum(1) == lat.N // 2]
    idx = (cfg.astype(np.int64) << (lat.N - 1 - np.arange(lat.N))).sum(-1)
    Hs = P.heisenberg_j1j2(lat.Lx, lat.Ly, lat.J1, lat.J2)[idx][:, idx]

    def energy(A_):
        psi = P.full_wavefunction(A_, lat)[idx]
        return float(psi @ (Hs @ psi) / (psi @ psi))
    rng = np.random.default_rng(2)
    Ad, Sd = _cuda(A), _cuda(S)
    Es = [energy(A)]
    for it in range(4):
        E, _ = peps.vmc_step(Ad, Sd, lat, _cuda(rng.random((8, 1024, 2))), _cuda(rng.random(A.shape)),
                             0.02, "f64")
        Es.append(energy(Ad.cpu().numpy()))
        _say(f"iteration {it}: sampled E {E[0].item():.4f}, exact after update {Es[-1]:.4f}")
    assert all(b < a for a, b in zip(Es, Es[1:])), Es
