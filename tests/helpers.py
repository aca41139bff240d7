"""Shared helpers of the GPU parity tests (inputs from synth, references from the oracle)."""
import numpy as np

import synth


def rel_inf(a, b):
    """max|a - b| / max|b| (b is the reference)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / (den if den > 0 else 1.0))


def smooth_inputs(shape, nt, nc=1, divfree=False, vtarget=None, seed=5):
    """(m_T, m_R, v*, w): smooth image, reference transported by v* (oracle), and a direction."""
    from oracle import transport as otr
    width = 0.6 * min(shape) ** 2 / 16.0
    mT = synth.smooth_image(shape, seed, width)
    if vtarget is None:
        vtarget = synth.cfl_literal_linf(max(shape), nt, 0.1)
    kmax = max(2, min(shape) // 8)
    vstar = synth.bandlimited_velocity(shape, seed + 70, kmax, vtarget, divfree=divfree, nc=nc,
                                       norm="linf")
    mR = otr.forward_only(mT, vstar, nt)
    w = synth.bandlimited_velocity(shape, seed + 90, kmax, vtarget, divfree=divfree, nc=nc, norm="linf")
    return mT, mR, vstar, w
