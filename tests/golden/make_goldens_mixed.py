"""Writes tests/golden/goldens_mixed.json: oracle values for the first configurations of
the 12x12 (D = 6, Dc = 36) and 16x16 (D = 8, Dc = 64) lattices of the mixed batch, and of
the 16x16, D = 6, Dc = 36 workload (amplitude, local energy, and log-derivatives at
seeded sample entries with the per-site Euler sums).

Calls only oracle/ and the seeded input generators; nothing here comes from the HIP path.

    python tests/golden/make_goldens_mixed.py
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

PLAN = (("mix_12x12_D6_Dc36", 2, 2, 0), ("16x16_D6_Dc36", 2, 1, 2), ("mix_16x16_D8_Dc64", 1, 0, 0))


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "goldens_mixed.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name, n_amp, n_e, n_grad in PLAN:
        if name in out:
            continue
        lat, A, S, _ = make_workload(name, n_amp)
        recs = []
        for b in range(n_amp):
            t0 = time.time()
            la, sg, fl = O.log_amplitude_one(A, lat, S[b])
            rec = {"index": b, "log_abs": la, "sign": int(sg), "flag": int(fl)}
            if b < n_e:
                rec["e_loc"] = O.local_energy_one(A, lat, S[b])
            if b < n_grad:
                d = O.log_derivative_one(A, lat, S[b]).reshape(lat.N, 2, -1)
                rng = np.random.default_rng(1000 + b)
                ent = []
                for _ in range(48):
                    m = int(rng.integers(lat.N))
                    s = int(S[b, m])
                    nz = np.nonzero(d[m, s])[0]
                    e = int(nz[rng.integers(nz.size)])
                    ent.append([m, s, e, float(d[m, s, e])])
                rec["grad_entries"] = ent
                rec["euler"] = [float(np.dot(A[m, int(S[b, m])].reshape(-1), d[m, int(S[b, m])])) for m in range(lat.N)]
            rec["oracle_seconds"] = round(time.time() - t0, 1)
            print(name, rec.get("log_abs"), rec.get("e_loc"), rec["oracle_seconds"], flush=True)
            recs.append(rec)
        out[name] = {"samples": recs}
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
