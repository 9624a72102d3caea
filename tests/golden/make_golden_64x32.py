"""Write tests/golden/oracle_64x32.json: oracle exponents on the 64x32^3 workload.

Calls only the oracle (the matrix-free C version).  The workload: 64x32^3 lattice,
8^4 Schwarz blocks, synthetic links exp(i 0.3 H) with seed [1211, 4], c_sw = 1,
antiperiodic time, kappa 0.1200 -> 0.1205 in N = 4 mass-interpolation steps (m linear),
complex Gaussian noise with seed [1214, 4, i, j].  Stored: the Schur-complement exponent
x_ij (difference form, all solves to 1e-13) of the first noise vector j = 0 of every
interpolation step i = 0..3, and of further noise vectors of the first step when asked.
An existing file is resumed and rewritten after every exponent (about 12 minutes each on
8 threads).

Run: python tests/golden/make_golden_64x32.py [n_first_step]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cref, dirac, estimator  # noqa: E402
from paper_1211_1214_amd import inputs  # noqa: E402

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_64x32.json")


def main(n_first=1):
    cfg = inputs.WORKLOADS["64x32^3"]
    lat, blk, n = cfg["lat"], cfg["blk"], cfg["n_interp"]
    out = json.load(open(PATH)) if os.path.exists(PATH) else {}
    if out.get("tol") != 1e-13:
        out = {}
    out.update({"workload": "64x32^3, blocks 8^4, eps 0.3 links seed [1211,4], c_sw 1, antiperiodic time, "
                            "kappa 0.1200->0.1205 in 4 steps linear in m, noise seed [1214,4,i,j]",
                "tol": 1e-13, "threads": cref.CRef.threads()})
    out.setdefault("x_schur", {})
    out.setdefault("seconds", {})
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    R = cref.CRef(U, lat, blk, cfg["csw"], -1)
    ms = estimator.interpolation_masses(dirac.mass(cfg["kappa1"]), dirac.mass(cfg["kappa2"]), n)
    todo = [(i, 0) for i in range(n)] + [(0, j) for j in range(1, n_first)]
    for i, j in todo:
        if f"{i},{j}" in out["x_schur"]:
            continue
        eta = inputs.make_noise(lat, cfg["seed"], i, j)
        t0 = time.time()
        x = R.exponent("schur", "diff", ms[i], ms[i + 1], eta, 1e-13)
        out["x_schur"][f"{i},{j}"] = x
        out["seconds"][f"{i},{j}"] = time.time() - t0
        print("schur", i, j, x, time.time() - t0, flush=True)
        with open(PATH, "w") as f:
            json.dump(out, f, indent=1)
    print("wrote", PATH)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1)
