"""Deformation gradient and det F_1 (FP64, CPU).

Paper: Appendix "Measures of Deformation Regularity", equation e:def-grad:
dt F + (v . grad) F = (grad v) F, F(0) = I, periodic, with det F_1 reported
(Tables t:defgrad-cinfty and t:defgrad-ut list its min, max, mean and spread).

Readings:
* (grad v)_{ik} = D_k v^i with the Nyquist-zeroed spectral derivative.
* Heun in time on the nodes t_j = j / n_t, like the state equation.
* Statistics are min, max, mean and population standard deviation of det F_1
  over the grid points, all in FP64.
* The paper equates det F_1 with det(grad y); the derivation gives
  det(grad y) = 1 / det F_1 for the pull-back map y = x - u_1. This module
  returns det F_1, the quantity the paper tabulates.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from . import spectral as sp
from .timebasis import velocity_at


def _rhs(F: np.ndarray, v: np.ndarray, gv: np.ndarray) -> np.ndarray:
    """-(v . grad) F + (grad v) F for F of shape (d, d, *grid)."""
    d = v.shape[0]
    out = np.zeros_like(F)
    for i in range(d):
        for j in range(d):
            gF = sp.grad(F[i, j])
            out[i, j] = -np.sum(v * gF, axis=0)
            for k in range(d):
                out[i, j] += gv[i, k] * F[k, j]
    return out


def _grad_v(v: np.ndarray) -> np.ndarray:
    """(grad v)[i, k] = D_k v^i."""
    return np.stack([sp.grad(v[i]) for i in range(v.shape[0])])


def deformation_gradient(vl: np.ndarray, nt: int) -> np.ndarray:
    """F_1 of shape (d, d, *grid) from a Heun solve of e:def-grad."""
    d = vl.shape[1]
    shape = vl.shape[2:]
    h = 1.0 / nt
    F = np.zeros((d, d) + tuple(shape))
    for i in range(d):
        F[i, i] = 1.0
    for j in range(nt):
        v0 = velocity_at(vl, j * h)
        v1 = velocity_at(vl, (j + 1) * h)
        k1 = _rhs(F, v0, _grad_v(v0))
        Fs = F + h * k1
        k2 = _rhs(Fs, v1, _grad_v(v1))
        F = F + 0.5 * h * (k1 + k2)
    return F


def det(F: np.ndarray) -> np.ndarray:
    """Pointwise determinant of a (d, d, *grid) tensor field (cofactor expansion)."""
    d = F.shape[0]
    if d == 2:
        return F[0, 0] * F[1, 1] - F[0, 1] * F[1, 0]
    return (F[0, 0] * (F[1, 1] * F[2, 2] - F[1, 2] * F[2, 1])
            - F[0, 1] * (F[1, 0] * F[2, 2] - F[1, 2] * F[2, 0])
            + F[0, 2] * (F[1, 0] * F[2, 1] - F[1, 1] * F[2, 0]))


def det_stats(vl: np.ndarray, nt: int) -> Tuple[np.ndarray, Tuple[float, float, float, float]]:
    """det F_1 and its (min, max, mean, std)."""
    J = det(deformation_gradient(vl, nt))
    return J, (float(J.min()), float(J.max()), float(J.mean()), float(J.std()))
