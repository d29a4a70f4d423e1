"""Seeded synthetic inputs for the PEPS amplitude / local-energy / log-derivative path.

This module only draws random numbers; it holds none of the method's arithmetic,
so both the HIP path and the CPU oracle can take their inputs from it.

Inputs follow the paper's problem statement (Sec. II-A): a PEPS on an open
Lx x Ly square lattice with physical dimension d = 2 and bond dimension D,
evaluated on spin configurations drawn one per Markov chain.  No trained PEPS
is available, so site tensors are i.i.d. Gaussian and configurations are
uniform over the S^z = 0 sector (the stand-in for |psi|^2 sampling).

Layouts (C order):
  A : float64 [N][2][D][D][D][D] = [site][phys][l][u][r][d], site m = i*Lx + j
  S : int8    [B][N], values {0, 1}; 0 is spin up (S^z = +1/2)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Lattice:
    Lx: int
    Ly: int
    D: int
    Dc: int
    J1: float = 1.0
    J2: float = 0.5

    @property
    def N(self) -> int:
        return self.Lx * self.Ly


@dataclass(frozen=True)
class Workload:
    """One named synthetic workload: lattice, tensor recipe, batch and seeds."""
    name: str
    lat: Lattice
    batch: int
    seed_A: int
    seed_S: int
    scaling: str        # "half": N(0,1) * 0.5 ; "frobenius": each site / ||A_m||_F
    precision: str      # GEMM precision the workload is quoted in: f64 | f32 | bf16


WORKLOADS = {
    # 4x4, D=2, Dc=4: exact regime (no cut exceeds D^2 = 4); all 2^16 configs enumerable.
    "4x4_D2_Dc4": Workload("4x4_D2_Dc4", Lattice(4, 4, 2, 4), 256, 1, 101, "half", "f64"),
    # 8x8, D=4, Dc=16, 4096 chains: the throughput workload.
    "8x8_D4_Dc16": Workload("8x8_D4_Dc16", Lattice(8, 8, 4, 16), 4096, 2, 102, "frobenius", "f32"),
    "16x16_D6_Dc36": Workload("16x16_D6_Dc36", Lattice(16, 16, 6, 36), 1024, 3, 103, "frobenius", "f32"),
    "24x24_D8_Dc64": Workload("24x24_D8_Dc64", Lattice(24, 24, 8, 64), 512, 4, 104, "frobenius", "bf16"),
    # the Dc proportional to D regime of the paper's single-core-group runs (D = 16, Dc = 32),
    # timed with variational boundary compression
    "16x16_D16_Dc32": Workload("16x16_D16_Dc32", Lattice(16, 16, 16, 32), 64, 5, 105, "frobenius", "f64"),
    # the three lattices of the mixed batch (2048 samples split 1024 / 614 / 410)
    "mix_8x8_D4_Dc16": Workload("mix_8x8_D4_Dc16", Lattice(8, 8, 4, 16), 1024, 51, 151, "frobenius", "f32"),
    "mix_12x12_D6_Dc36": Workload("mix_12x12_D6_Dc36", Lattice(12, 12, 6, 36), 614, 52, 152, "frobenius", "f32"),
    "mix_16x16_D8_Dc64": Workload("mix_16x16_D8_Dc64", Lattice(16, 16, 8, 64), 410, 53, 153, "frobenius", "f32"),
}

# the mixed batch: (workload, samples) in its 50/30/20 split of 2048
MIXED_BATCH = (("mix_8x8_D4_Dc16", 1024), ("mix_12x12_D6_Dc36", 614), ("mix_16x16_D8_Dc64", 410))


def make_tensors(lat: Lattice, seed: int, scaling: str) -> np.ndarray:
    """Site tensors A[site][phys][l][u][r][d], float64, i.i.d. N(0,1) then scaled."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((lat.N, 2, lat.D, lat.D, lat.D, lat.D))
    if scaling == "half":
        A *= 0.5
    elif scaling == "frobenius":
        nrm = np.sqrt((A.reshape(lat.N, -1) ** 2).sum(axis=1))
        A /= nrm[:, None, None, None, None, None]
    else:
        raise ValueError(f"unknown scaling {scaling!r}")
    return np.ascontiguousarray(A)


def make_configs(lat: Lattice, batch: int, seed: int) -> np.ndarray:
    """S[b] = random permutation of ceil(N/2) zeros and floor(N/2) ones, int8
    (the S^z = 0 sector for even N, S^z = +1/2 for odd N)."""
    rng = np.random.default_rng(seed)
    base = np.zeros(lat.N, dtype=np.int8)
    base[lat.N - lat.N // 2:] = 1
    S = np.empty((batch, lat.N), dtype=np.int8)
    for b in range(batch):
        S[b] = rng.permutation(base)
    return S


def make_workload(name: str, batch: int | None = None):
    """(lattice, A, S, precision) for a named workload; `batch` may shrink it."""
    w = WORKLOADS[name]
    B = w.batch if batch is None else batch
    A = make_tensors(w.lat, w.seed_A, w.scaling)
    S = make_configs(w.lat, max(B, 0), w.seed_S)
    return w.lat, A, S, w.precision


def make_random(lat: Lattice, batch: int, seed: int, scaling: str = "frobenius"):
    """Ad-hoc lattice with seeded tensors and S^z = 0 configurations."""
    return make_tensors(lat, seed, scaling), make_configs(lat, batch, seed + 1000)
