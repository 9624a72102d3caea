"""Write tests/golden/oracle_32x16.json: oracle exponents on the 32x16^3 workload (the
differentiation workload).

Calls only the oracle (the matrix-free C version for the solves, oracle.estimator for the
combination).  The workload: 32x16^3 lattice, 4^4 Schwarz blocks, synthetic links exp(i 0.3 H)
with seed [1211, 5], c_sw = 1, antiperiodic time, kappa 0.1200 -> 0.1205, complex Gaussian
noise with seed [1214, 5, 0, j], N_hit = 8.  Stored: every Schur-complement exponent x_0j
(difference form, all solves to 1e-13) and log W_gl of Eq. (8).

Run: python tests/golden/make_golden_32x16.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cref, dirac, estimator  # noqa: E402
from paper_1211_1214_amd import inputs  # noqa: E402

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_32x16.json")


def main():
    cfg = inputs.WORKLOADS["32x16^3"]
    lat, blk, nhit = cfg["lat"], cfg["blk"], cfg["n_hit"]
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    R = cref.CRef(U, lat, blk, cfg["csw"], -1)
    m1, m2 = dirac.mass(cfg["kappa1"]), dirac.mass(cfg["kappa2"])
    out = {"workload": "32x16^3, blocks 4^4, eps 0.3 links seed [1211,5], c_sw 1, antiperiodic time, "
                       "kappa 0.1200->0.1205, noise seed [1214,5,0,j]",
           "tol": 1e-13, "threads": cref.CRef.threads(), "x_schur": {}}
    for j in range(nhit):
        eta = inputs.make_noise(lat, cfg["seed"], 0, j)
        t0 = time.time()
        out["x_schur"][str(j)] = R.exponent("schur", "diff", m1, m2, eta, 1e-13)
        print("schur", j, out["x_schur"][str(j)], time.time() - t0, flush=True)
    x = np.array([[out["x_schur"][str(j)] for j in range(nhit)]])
    out["log_w_gl"] = estimator.log_w_gl(x)
    with open(PATH, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", PATH)


if __name__ == "__main__":
    main()
