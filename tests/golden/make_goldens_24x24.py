"""Writes tests/golden/goldens_24x24_D8_Dc64.json: oracle values for the first configurations
of the 24x24, D = 8, Dc = 64 workload (seeded inputs from paper_1806_03761_amd.workloads).

Calls only oracle/ (the FP64 CPU oracle) and the seeded input generators; nothing here
comes from the HIP path.  Run from the repository root:

    python tests/golden/make_goldens_24x24.py [n_amplitude] [n_energy]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1806_03761_amd.workloads import make_workload  # noqa: E402


def main():
    n_amp = int(sys.argv[1]) if len(sys.argv) > 1 else 3
    n_e = int(sys.argv[2]) if len(sys.argv) > 2 else 1
    name = "24x24_D8_Dc64"
    lat, A, S, _ = make_workload(name, max(n_amp, n_e))
    out = {"workload": name, "seed_A": 4, "seed_S": 104, "samples": []}
    for b in range(max(n_amp, n_e)):
        t0 = time.time()
        la, sg, fl = O.log_amplitude_one(A, lat, S[b])
        rec = {"index": b, "log_abs": la, "sign": int(sg), "flag": int(fl)}
        if b < n_e:
            rec["e_loc"] = O.local_energy_one(A, lat, S[b])
        rec["oracle_seconds"] = round(time.time() - t0, 1)
        out["samples"].append(rec)
        print(rec, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "goldens_24x24_D8_Dc64.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
