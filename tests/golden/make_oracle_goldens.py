"""Writes the stored expected values of the full-size GPU tests that the FP64
oracle is too slow to recompute inside a test.  Calls only oracle/ (and the
input generators); run from the repository root:

    python tests/golden/make_oracle_goldens.py
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ccmf_oracle as O  # noqa: E402
from paper_2103_05968_amd import microstructures as M  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def spheres32_f64():
    cfg = M.CONFIGS["c1"]
    t = time.time()
    r = O.admm_solve(M.config_c1(), cfg["loads"][0], tol=cfg["tol"], max_iter=100000)
    return {
        "what": "FP64 oracle (damped ADMM of Sec. 3.2, readings of the design notes) on the 32^3 sphere workload: "
                "overlapping spheres r = 4, 15 %, kappa 0.3 / 1, seed 1, load e1, tol 1e-6",
        "grid": list(cfg["dims"]), "load": list(cfg["loads"][0]), "tol": cfg["tol"],
        "geff": r.geff, "iterations": r.iterations, "converged": r.converged,
        "dual_est": r.dual_est, "mean_flux": r.mean_flux.tolist(), "seconds": round(time.time() - t, 1),
    }


if __name__ == "__main__":
    out = spheres32_f64()
    with open(os.path.join(HERE, "oracle_spheres32_f64.json"), "w") as f:
        json.dump(out, f, indent=2)
    print(out)
