"""RK2 (Heun) transport solves of the optimality systems (FP64, CPU).

Paper: the state equation e:first-order-forward (dt m + grad m . v = 0,
m(0) = m_T), the adjoint equation e:first-order-adjoint (-dt lambda -
div(v lambda) = 0, lambda(1) = m_R - m_1), the Gauss-Newton incremental
equations e:gauss-newton (incremental state with forcing grad m . v~ and
m~(0) = 0; incremental adjoint without the lambda term, lambda~(1) = -m~_1),
Section "Numerical Discretization" (explicit RK2 in time, h_t = 1/n_t) and
Algorithm a:hessian-matvec (incremental forward then incremental adjoint solve).

Readings where the paper is silent:
* RK2 is Heun's method (explicit trapezoid) on nodes t_j = j h, h = 1/n_t.
* The adjoint is stepped backward with Heun on the conservative form, using
  v(t_{j+1}) in the first stage and v(t_j) in the second. With the
  Nyquist-zeroed derivative this step is exactly the transpose of the forward
  step, so the optimise-then-discretise adjoint is also the discrete adjoint.
* The time integral of the body force b_l(t) lambda grad m is taken with the
  quadrature that Heun's adjoint induces:
      sum_j (h/2) [ b_l(t_j) lambda*_j grad m^j + b_l(t_{j+1}) lambda^{j+1} grad m*_j ]
  where m*_j is the state's first-stage value and lambda*_j the adjoint's. It is
  second-order consistent with the integral and makes the gradient exact for
  the discrete objective.
* The incremental state uses the stage value m*_j in its second-stage forcing
  (-v~(t_{j+1}) . grad m*_j), the exact linearisation of the state step.

All fields are FP64 NumPy arrays; velocities are coefficient arrays of shape
(n_c, d, *grid).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

from . import spectral as sp
from .timebasis import basis_values, velocity_at


@dataclass
class Trajectory:
    """What a forward solve leaves for the adjoint and the Hessian matvec.

    grad_m[j]  = grad m^j       (state at t_j),           j = 0..nt-1
    grad_ms[j] = grad m*_j      (first Heun stage value), j = 0..nt-1
    """
    m1: np.ndarray
    grad_m: List[np.ndarray]
    grad_ms: List[np.ndarray]


def _dot(v: np.ndarray, g: np.ndarray) -> np.ndarray:
    return np.sum(v * g, axis=0)


def forward_state(mT: np.ndarray, vl: np.ndarray, nt: int) -> Trajectory:
    """Heun solve of dt m + v . grad m = 0 from m(0) = m_T; keeps the gradients."""
    h = 1.0 / nt
    m = mT.copy()
    gm_list, gms_list = [], []
    for j in range(nt):
        v0 = velocity_at(vl, j * h)
        v1 = velocity_at(vl, (j + 1) * h)
        gm = sp.grad(m)
        r1 = -_dot(v0, gm)
        ms = m + h * r1
        gms = sp.grad(ms)
        r2 = -_dot(v1, gms)
        gm_list.append(gm)
        gms_list.append(gms)
        m = m + 0.5 * h * (r1 + r2)
    return Trajectory(m, gm_list, gms_list)


def forward_only(mT: np.ndarray, vl: np.ndarray, nt: int) -> np.ndarray:
    """m_1 from the same Heun solve, without keeping the trajectory."""
    h = 1.0 / nt
    m = mT.copy()
    for j in range(nt):
        v0 = velocity_at(vl, j * h)
        v1 = velocity_at(vl, (j + 1) * h)
        r1 = -_dot(v0, sp.grad(m))
        ms = m + h * r1
        r2 = -_dot(v1, sp.grad(ms))
        m = m + 0.5 * h * (r1 + r2)
    return m


def adjoint_step(lam: np.ndarray, v0: np.ndarray, v1: np.ndarray, h: float
                 ) -> Tuple[np.ndarray, np.ndarray]:
    """One backward Heun step of -dt lam - div(v lam) = 0 from t_{j+1} to t_j.

    Returns (lam^j, lam*_j).
    """
    s1 = sp.div(v1 * lam)
    lams = lam + h * s1
    s2 = sp.div(v0 * lams)
    return lam + 0.5 * h * (s1 + s2), lams


def adjoint_with_force(lam1: np.ndarray, vl: np.ndarray, traj: Trajectory, nt: int
                       ) -> Tuple[np.ndarray, np.ndarray]:
    """Backward adjoint solve from lam(1) = lam1, accumulating the body force.

    Returns (lam^0, F) with F of shape (nc, d, *grid):
    F_l = sum_j (h/2) [ b_l(t_j) lam*_j grad m^j + b_l(t_{j+1}) lam^{j+1} grad m*_j ].
    Used with lam1 = m_R - m_1 for the reduced gradient and with
    lam1 = -m~_1 for the Gauss-Newton Hessian matvec.
    """
    h = 1.0 / nt
    nc = vl.shape[0]
    lam = lam1.copy()
    F = np.zeros_like(vl)
    for j in range(nt - 1, -1, -1):
        v0 = velocity_at(vl, j * h)
        v1 = velocity_at(vl, (j + 1) * h)
        b0 = basis_values(nc, j * h)
        b1 = basis_values(nc, (j + 1) * h)
        lam_next, lams = adjoint_step(lam, v0, v1, h)
        for l in range(nc):
            F[l] += 0.5 * h * (b0[l] * lams * traj.grad_m[j] + b1[l] * lam * traj.grad_ms[j])
        lam = lam_next
    return lam, F


def incremental_state(vl: np.ndarray, vtl: np.ndarray, traj: Trajectory, nt: int) -> np.ndarray:
    """Heun solve of dt m~ + v . grad m~ + v~ . grad m = 0 from m~(0) = 0; returns m~_1."""
    h = 1.0 / nt
    mt = np.zeros(traj.m1.shape)
    for j in range(nt):
        v0 = velocity_at(vl, j * h)
        v1 = velocity_at(vl, (j + 1) * h)
        w0 = velocity_at(vtl, j * h)
        w1 = velocity_at(vtl, (j + 1) * h)
        r1 = -_dot(v0, sp.grad(mt)) - _dot(w0, traj.grad_m[j])
        mts = mt + h * r1
        r2 = -_dot(v1, sp.grad(mts)) - _dot(w1, traj.grad_ms[j])
        mt = mt + 0.5 * h * (r1 + r2)
    return mt
