"""Write tests/golden/oracle_48x24.json: oracle exponents on the 48x24^3 workload.

Calls only the oracle (the matrix-free C version).  The workload: 48x24^3 lattice,
6^4 Schwarz blocks, synthetic links exp(i 0.3 H) with seed [1211, 3], c_sw = 1,
antiperiodic time, kappa 0.1200 -> 0.1205, complex Gaussian noise with seed
[1214, 3, 0, j].  Stored: the Schur-complement exponent x_0j (difference form, all
solves to 1e-13) for the first noise vectors, the full-operator exponent for j = 0,
and the iteration counts of the oracle's own solves for one Schur exponent (used to
scale the benchmark's bounded CPU sample to one estimate).

Run: python tests/golden/make_golden_48x24.py [n_schur]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cref, dirac  # noqa: E402
from paper_1211_1214_amd import inputs  # noqa: E402


def main(n_schur=2):
    cfg = inputs.WORKLOADS["48x24^3"]
    lat, blk = cfg["lat"], cfg["blk"]
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    R = cref.CRef(U, lat, blk, cfg["csw"], -1)
    m1, m2 = dirac.mass(cfg["kappa1"]), dirac.mass(cfg["kappa2"])
    out = {"workload": "48x24^3, blocks 6^4, eps 0.3 links seed [1211,3], c_sw 1, antiperiodic time, "
                       "kappa 0.1200->0.1205, noise seed [1214,3,0,j]",
           "tol": 1e-13, "x_schur": {}, "x_full": {}, "threads": cref.CRef.threads()}
    for j in range(n_schur):
        eta = inputs.make_noise(lat, cfg["seed"], 0, j)
        t0 = time.time()
        x, iters, secs = R.exponent_recorded("schur", "diff", m1, m2, eta, 1e-13)
        out["x_schur"][str(j)] = x
        if j == 0:
            out["schur_solve_iterations"] = iters
            out["schur_solve_seconds"] = secs
            out["schur_seconds"] = time.time() - t0
        print("schur", j, x, iters, time.time() - t0, flush=True)
    eta = inputs.make_noise(lat, cfg["seed"], 0, 0)
    x, iters, secs = R.exponent_recorded("full", "diff", m1, m2, eta, 1e-13)
    out["x_full"]["0"] = x
    out["full_solve_iterations"] = iters
    print("full", x, iters, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_48x24.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2)
