"""Writes c2lit_solve.json: the FP64 oracle's beta-continuation solve of the 512^2, nt = 32
headline workload (H2, beta 1e-1 -> 1e-4, relative gradient 1e-3 per level against the first
level's ||g_0||_inf). Calls only the oracle and the seeded input generators; takes a few
minutes on the CPU.

    python tests/golden/make_c2lit_solve.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import krylov as okr  # noqa: E402
from oracle import reduced as ord_  # noqa: E402
from oracle import transport as otr  # noqa: E402


def main() -> None:
    spec = synth.CONFIGS["c2lit"]
    mT, vstar = synth.make_inputs(spec)
    mR = otr.forward_only(mT, vstar, spec.nt)
    P = ord_.Problem(mT, mR, spec.nt, 1, spec.reg, 0, spec.beta_levels[0])
    t0 = time.time()
    v, reps = okr.continuation(P, spec.beta_levels, gtol=1e-3, max_outer=50)
    m1 = otr.forward_only(mT, v, spec.nt)
    mis = float(np.sum((m1 - mR) ** 2) / np.sum((mT - mR) ** 2))
    out = {
        "source": "FP64 oracle (oracle.krylov.continuation) on the synthetic 512^2 nt = 32 workload "
                  "'c2lit'; written by tests/golden/make_c2lit_solve.py",
        "beta_levels": list(spec.beta_levels),
        "gtol": 1e-3,
        "relative_mismatch": mis,
        "levels": [{"beta": b, "iterations": r.iterations, "cg_iterations": int(sum(r.cg_iterations)),
                    "converged": bool(r.converged)} for b, r in zip(spec.beta_levels, reps)],
        "J_dist": float(ord_.objective(ord_.Problem(mT, mR, spec.nt, 1, spec.reg, 0, spec.beta_levels[-1]), v)[1]),
        "v_l2": float(np.sqrt(np.sum(v ** 2))),
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2lit_solve.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
