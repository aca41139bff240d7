"""Chebyshev expansion of the velocity in time (FP64, CPU).

Paper: Section "Spectral Galerkin Method" (equation e:expansion,
v(x, t) = sum_{l=1}^{n_c} b_l(t) v_l(x)) and Appendix "Expansion in Time:
Derivation" (Chebyshev polynomials as b_l; regulariser weights c_ll').

Readings:
* b_l(t) = T_{l-1}(2t - 1), the Chebyshev polynomial of degree l-1 shifted to
  [0, 1], evaluated directly at the time nodes t_j = j / n_t (modal
  coefficients; the Gauss-Lobatto nodes the appendix mentions play no role).
* The appendix states c_ll' = delta_ll'. For unit weight on [0, 1] that is not
  the Gram matrix of the shifted Chebyshev polynomials, but it is what the
  paper says its scheme uses, so the regulariser is (beta/2) sum_l <v_l, A v_l>.
"""
from __future__ import annotations

import numpy as np


def cheb_T(n: int, s: float) -> float:
    """T_n(s) by the three-term recurrence T_0 = 1, T_1 = s, T_{n+1} = 2 s T_n - T_{n-1}."""
    if n == 0:
        return 1.0
    t0, t1 = 1.0, s
    for _ in range(n - 1):
        t0, t1 = t1, 2.0 * s * t1 - t0
    return t1


def basis(l: int, t: float) -> float:
    """b_l(t) = T_{l-1}(2 t - 1) for l = 1..n_c (the code uses 0-based l-1)."""
    return cheb_T(l, 2.0 * t - 1.0)


def basis_values(nc: int, t: float) -> np.ndarray:
    """[b_1(t), .., b_nc(t)]."""
    return np.array([basis(l, t) for l in range(nc)])


def velocity_at(vl: np.ndarray, t: float) -> np.ndarray:
    """v(t) = sum_l b_l(t) v_l for coefficients vl of shape (nc, d, *grid)."""
    b = basis_values(vl.shape[0], t)
    out = np.zeros(vl.shape[1:])
    for l in range(vl.shape[0]):
        out += b[l] * vl[l]
    return out
