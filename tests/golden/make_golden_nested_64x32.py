"""Write tests/golden/oracle_nested_64x32.json: nested-DD exponents on the 64x32^3 workload.

Calls only the oracle (the matrix-free C version through oracle.nested.NestedMatrixFree).
The workload: 64x32^3 lattice, links exp(i 0.3 H) with seed [1211, 4], c_sw = 1,
antiperiodic time, outer blocks 8^4 split into inner blocks 4^4 (Sec. 2.2), kappa
0.1200 -> 0.1205 in N = 4 mass-interpolation steps (m linear).  For each outer colour c
the noise of the nested factor is complex Gaussian with seed [1214, 40 + c, i, j].
Stored: the exponent x_ij (difference form, all solves to 1e-13) of the first step i = 0
for the first noise vectors j, per colour.

Run: python tests/golden/make_golden_nested_64x32.py [n_first_step]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cref, dirac, estimator  # noqa: E402
from oracle.nested import NestedMatrixFree  # noqa: E402
from paper_1211_1214_amd import inputs  # noqa: E402

INNER = (4, 4, 4, 4)


def main(n_first=1):
    cfg = inputs.WORKLOADS["64x32^3"]
    lat, blk, n = cfg["lat"], cfg["blk"], cfg["n_interp"]
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    ms = estimator.interpolation_masses(dirac.mass(cfg["kappa1"]), dirac.mass(cfg["kappa2"]), n)
    out = {"workload": "64x32^3, outer blocks 8^4, inner blocks 4^4, eps 0.3 links seed [1211,4], c_sw 1, "
                       "antiperiodic time, kappa 0.1200->0.1205 in 4 steps linear in m, "
                       "noise seed [1214,40+colour,i,j]",
           "tol": 1e-13, "inner_blocks": list(INNER), "x_nested": {}, "threads": cref.CRef.threads(),
           "seconds": {}}
    for c in (0, 1):
        R = NestedMatrixFree(U, lat, blk, INNER, cfg["csw"], c, -1, 1e-13)
        for j in range(n_first):
            eta = inputs.make_noise(lat, 40 + c, 0, j)
            t0 = time.time()
            x = estimator.x_schur_diff(R, ms[0], ms[1], eta)
            out["x_nested"][f"{c},0,{j}"] = x
            out["seconds"][f"{c},0,{j}"] = time.time() - t0
            print("nested", c, 0, j, x, time.time() - t0, flush=True)
        R.close()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_nested_64x32.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1)
