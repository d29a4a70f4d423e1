"""Writes tests/golden/var_<workload>_<kind>_<index>.json: the oracle's result for one
configuration with the variational boundary compression (one sweep), and its own rounding
noise.

W(S) is linear in every site tensor (the compression is homogeneous in the applied row),
so scaling site m by (1 + d_m), |d_m| <= 2^-30, multiplies W exactly by prod_m (1 + d_m)
and leaves every ratio W(S')/W(S), hence E(S), unchanged.  What else moves is rounding:
  amp:  |ln|W|(scaled) - ln|W| - sum_m ln(1 + d_m)|, the largest over two seeds;
  eloc: |E(scaled) - E|, one seed.

Calls only oracle/ and the seeded input generators.  Run from the repository root:

    python tests/golden/make_goldens_variational.py <workload> <index> <amp|eloc>
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1806_03761_amd.workloads import make_workload  # noqa: E402

SWEEPS = 1


def main():
    name, b, kind = sys.argv[1], int(sys.argv[2]), sys.argv[3]
    lat, A, S, _ = make_workload(name, b + 1)
    s = S[b]
    t0 = time.time()
    out = {"workload": name, "index": b, "kind": kind, "sweeps": SWEEPS, "config": s.tolist()}
    if kind == "amp":
        la, sg, fl = O.log_amplitude_one(A, lat, s, SWEEPS)
        out.update(log_abs=la, sign=int(sg), flag=int(fl))
        noise = 0.0
        for k in (1, 2):
            d = np.random.default_rng(7200 + 10 * b + k).uniform(-1.0, 1.0, size=lat.N) * 2.0 ** -30
            la2 = O.log_amplitude_one(A * (1.0 + d)[:, None, None, None, None, None], lat, s, SWEEPS)[0]
            noise = max(noise, abs(la2 - float(np.sum(np.log1p(d))) - la))
        out["noise"] = noise
    else:
        e = O.local_energy_one(A, lat, s, sweeps=SWEEPS)
        d = np.random.default_rng(7300 + b).uniform(-1.0, 1.0, size=lat.N) * 2.0 ** -30
        e2 = O.local_energy_one(A * (1.0 + d)[:, None, None, None, None, None], lat, s, sweeps=SWEEPS)
        out.update(e_loc=e, noise=abs(e2 - e))
    out["oracle_seconds"] = round(time.time() - t0, 1)
    print({k: v for k, v in out.items() if k != "config"}, flush=True)
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, f"var_{name}_{kind}_{b}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
