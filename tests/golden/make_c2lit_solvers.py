"""Writes c2lit_solvers.json: the FP64 oracle's GN-PCG solve and globalised Picard iteration
(with and without the objective-stagnation stop) on the 512^2, nt = 32, H2 workload 'c2lit'
at beta = 1e-2, from v = 0 to a relative gradient of 1e-3. Calls only the oracle and the
seeded input generators; takes several minutes on the CPU.

    python tests/golden/make_c2lit_solvers.py
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


def summary(rep, seconds):
    return {"outer_iterations": rep.iterations, "matvecs": int(sum(rep.cg_iterations)), "n_pde": rep.n_pde,
            "converged": bool(rep.converged), "grad_rel": float(rep.gnorm_inf[-1] / rep.gnorm0_inf),
            "J": float(rep.J[-1]), "seconds": seconds}


def main() -> None:
    spec = synth.CONFIGS["c2lit"]
    beta = 1e-2
    mT, vstar = synth.make_inputs(spec)
    mR = otr.forward_only(mT, vstar, spec.nt)
    P = ord_.Problem(mT, mR, spec.nt, 1, spec.reg, 0, beta)
    out = {"source": "FP64 oracle (oracle.krylov.gauss_newton, oracle.krylov.picard) on the synthetic 512^2 "
                     "nt = 32 workload 'c2lit' at beta = 1e-2; written by tests/golden/make_c2lit_solvers.py",
           "beta": beta, "gtol": 1e-3}
    t0 = time.time()
    _, rep, _ = okr.gauss_newton(P, np.zeros(P.vshape()), gtol=1e-3, max_outer=50)
    out["gn_pcg"] = summary(rep, time.time() - t0)
    t0 = time.time()
    _, rep, _ = okr.picard(P, np.zeros(P.vshape()), gtol=1e-3, max_outer=2000)
    out["picard"] = summary(rep, time.time() - t0)
    t0 = time.time()
    _, rep, _ = okr.picard(P, np.zeros(P.vshape()), gtol=1e-3, max_outer=2000, stagnation=(10 ** 9, 0.0))
    out["picard_no_stagnation_stop"] = summary(rep, time.time() - t0)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2lit_solvers.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
