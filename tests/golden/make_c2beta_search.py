"""Writes c2beta_search.json: the FP64 oracle's beta search bounded by det F_1 on the 256^2,
nt = 64, H1 workload 'c2beta' (decade descent from beta = 1, then bisection; relative
gradient 1e-3 per solve). The reference image is the oracle's forward solve of the seeded
velocity. Calls only the oracle and the seeded input generators; takes a few minutes on the
CPU.

    python tests/golden/make_c2beta_search.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import krylov as okr  # noqa: E402
from oracle import reduced as ord_  # noqa: E402
from oracle import transport as otr  # noqa: E402


def main() -> None:
    spec = synth.CONFIGS["c2beta"]
    eps = spec.extra["eps_F"]
    mT, vstar = synth.make_inputs(spec)
    mR = otr.forward_only(mT, vstar, spec.nt)
    P = ord_.Problem(mT, mR, spec.nt, 1, spec.reg, 0, 1.0)
    t0 = time.time()
    _, rep = okr.beta_search(P, eps, gtol=1e-3, max_outer=50)
    out = {
        "source": "FP64 oracle (oracle.krylov.beta_search) on the synthetic 256^2 nt = 64 workload "
                  "'c2beta'; written by tests/golden/make_c2beta_search.py",
        "eps_F": eps,
        "gtol": 1e-3,
        "trials": [{"beta": t.beta, "min_det": t.min_det, "l2_rel": t.l2_rel, "accepted": bool(t.accepted)}
                   for t in rep.trials],
        "beta_star": rep.beta_star,
        "min_det_star": rep.min_det_star,
        "dbeta_min": rep.dbeta_min,
        "breached": bool(rep.breached),
        "reason": rep.reason,
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2beta_search.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
