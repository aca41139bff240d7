"""Writes c2lit_newton_solve.json: the FP64 oracle's beta continuation with the full-Newton
Hessian on the 512^2, nt = 32, H2 workload 'c2lit' (beta 1e-1 -> 1e-4, relative gradient 1e-3
per level against the first level's ||g_0||_inf, each level warm-started). Calls only the
oracle and the seeded input generators; takes several minutes on the CPU.

    python tests/golden/make_c2lit_newton_solve.py
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
    t0 = time.time()
    v = np.zeros((1, 2) + tuple(spec.shape))
    gref = None
    levels = []
    for b in spec.beta_levels:
        Pb = ord_.Problem(mT, mR, spec.nt, 1, spec.reg, 0, b)
        v, rep, _ = okr.gauss_newton(Pb, v, gtol=1e-3, max_outer=50, gref_inf=gref, hessian="newton")
        if gref is None:
            gref = rep.gnorm0_inf
        levels.append({"beta": b, "iterations": rep.iterations, "cg_iterations": int(sum(rep.cg_iterations)),
                       "converged": bool(rep.converged)})
    m1 = otr.forward_only(mT, v, spec.nt)
    out = {
        "source": "FP64 oracle (oracle.krylov.gauss_newton, hessian='newton', warm-started per level) on the "
                  "synthetic 512^2 nt = 32 workload 'c2lit'; written by tests/golden/make_c2lit_newton_solve.py",
        "beta_levels": list(spec.beta_levels),
        "gtol": 1e-3,
        "relative_mismatch": float(np.sum((m1 - mR) ** 2) / np.sum((mT - mR) ** 2)),
        "levels": levels,
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2lit_newton_solve.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
