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


def adjoint_trajectory(lam1: np.ndarray, vl: np.ndarray, nt: int) -> List[Tuple[np.ndarray, np.ndarray]]:
    """The adjoint states of the gradient's backward solve from lam(1) = lam1:
    entry j is (lam^{j+1}, lam*_j), j = 0..nt-1 (what the full-Newton matvec reads)."""
    h = 1.0 / nt
    out: List[Tuple[np.ndarray, np.ndarray]] = [None] * nt
    lam = lam1.copy()
    for j in range(nt - 1, -1, -1):
        lam_next, lams = adjoint_step(lam, velocity_at(vl, j * h), velocity_at(vl, (j + 1) * h), h)
        out[j] = (lam.copy(), lams)
        lam = lam_next
    return out


def incremental_state_trajectory(vl: np.ndarray, vtl: np.ndarray, traj: Trajectory, nt: int
                                 ) -> Tuple[np.ndarray, List[np.ndarray], List[np.ndarray]]:
    """incremental_state that also keeps grad m~^j and grad m~*_j, j = 0..nt-1."""
    h = 1.0 / nt
    mt = np.zeros(traj.m1.shape)
    g_list, gs_list = [], []
    for j in range(nt):
        v0 = velocity_at(vl, j * h)
        v1 = velocity_at(vl, (j + 1) * h)
        w0 = velocity_at(vtl, j * h)
        w1 = velocity_at(vtl, (j + 1) * h)
        gmt = sp.grad(mt)
        r1 = -_dot(v0, gmt) - _dot(w0, traj.grad_m[j])
        mts = mt + h * r1
        gmts = sp.grad(mts)
        r2 = -_dot(v1, gmts) - _dot(w1, traj.grad_ms[j])
        g_list.append(gmt)
        gs_list.append(gmts)
        mt = mt + 0.5 * h * (r1 + r2)
    return mt, g_list, gs_list


def newton_adjoint_with_force(lamt1: np.ndarray, vl: np.ndarray, vtl: np.ndarray, traj: Trajectory,
                              adj: List[Tuple[np.ndarray, np.ndarray]], grad_mt: List[np.ndarray],
                              grad_mts: List[np.ndarray], nt: int) -> np.ndarray:
    """Full-Newton incremental adjoint (e:sec-order-iadj) with its body force.

    The second variations keep the terms in lambda that the Gauss-Newton system
    drops: the incremental adjoint -dt lam~ - div(v lam~) - div(v~ lam) = 0 from
    lam~(1) = -m~_1, and the incremental body force f~ = lam~ grad m + lam grad m~.
    Discretised as the directional derivative of the gradient's Heun-adjoint step
    and quadrature (so that the matvec is the exact Hessian of the discrete
    objective): with lam = lam^{j+1}, lam* = lam*_j of the gradient's solve,
        s1~ = div(v(t_{j+1}) lam~ + v~(t_{j+1}) lam),   lam~* = lam~ + h s1~,
        s2~ = div(v(t_j) lam~* + v~(t_j) lam*),         lam~ <- lam~ + h/2 (s1~ + s2~),
        F~_l += (h/2) [ b_l(t_j) (lam~* grad m^j + lam* grad m~^j)
                        + b_l(t_{j+1}) (lam~ grad m*_j + lam grad m~*_j) ].
    """
    h = 1.0 / nt
    nc = vl.shape[0]
    lt = lamt1.copy()
    F = np.zeros_like(vl)
    for j in range(nt - 1, -1, -1):
        v0 = velocity_at(vl, j * h)
        v1 = velocity_at(vl, (j + 1) * h)
        w0 = velocity_at(vtl, j * h)
        w1 = velocity_at(vtl, (j + 1) * h)
        b0 = basis_values(nc, j * h)
        b1 = basis_values(nc, (j + 1) * h)
        lam, lams = adj[j]
        s1 = sp.div(v1 * lt + w1 * lam)
        lts = lt + h * s1
        s2 = sp.div(v0 * lts + w0 * lams)
        for l in range(nc):
            F[l] += 0.5 * h * (b0[l] * (lts * traj.grad_m[j] + lams * grad_mt[j])
                               + b1[l] * (lt * traj.grad_ms[j] + lam * grad_mts[j]))
        lt = lt + 0.5 * h * (s1 + s2)
    return F

