"""Objective, reduced gradient and Gauss-Newton Hessian matvec (FP64, CPU).

Paper: the objective (e:objective with the quadratic regulariser
e:quadratic-regularization), the reduced gradient g = beta A v + gamma grad p + f
with body force f = lambda grad m (e:first-order-control) and its eliminated
form g^ = beta A v + K[f] (e:eliminated-control), the GN reduced Hessian
H v~ = beta A v~ + K[f~] with f~ = lambda~ grad m (e:gauss-newton,
e:eliminated-icontrol), Algorithm a:hessian-matvec, and the expansion in time
(e:control-equation-expansion, e:incremental-control-equation-expansion with
c_ll' = delta_ll').

Readings:
* J^h = (h_d / 2) sum_x (m_R - m_1)^2 + (beta / 2) sum_l <v_l, A v_l>_h, with
  <a, b>_h = h_d sum a b and h_d = prod(2 pi / N_i).
* g and H v~ are the nodal values of the L2-Riesz representatives (no h_d
  factor): dJ = <g, dv>_h. Table t:eigenvalues (H's largest eigenvalue equal to
  beta max a(k) at beta = 1e6) fixes this scaling.
* K acts on the body force only (gamma = 1); beta A v is never projected.
  Table t:eigenvalues (Stokes, beta = 1e-3: smallest eigenvalue exactly
  1e-3 = beta * a(k) at |k| = 1, the curl-free modes) fixes this.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

from . import spectral as sp
from . import transport as tr


@dataclass
class Problem:
    """One registration problem: images, discretisation and regulariser."""
    mT: np.ndarray
    mR: np.ndarray
    nt: int
    nc: int = 1
    reg: int = 1          # 1: H1 (A = -Lap), 2: H2 (A = Lap^2)
    gamma: int = 0        # 1: incompressible, K applied to body forces
    beta: float = 1e-2

    @property
    def shape(self) -> Tuple[int, ...]:
        return self.mT.shape

    @property
    def d(self) -> int:
        return self.mT.ndim

    @property
    def hd(self) -> float:
        return sp.cell_volume(self.shape)

    def vshape(self) -> Tuple[int, ...]:
        return (self.nc, self.d) + tuple(self.shape)

    def inner(self, a: np.ndarray, b: np.ndarray) -> float:
        """<a, b>_h over all coefficients, components and grid points."""
        return self.hd * float(np.sum(a * b))

    def project(self, f: np.ndarray) -> np.ndarray:
        """K applied to each coefficient's vector field if gamma = 1, else identity."""
        if not self.gamma:
            return f
        return np.stack([sp.apply_K(f[l]) for l in range(f.shape[0])])

    def reg_energy(self, vl: np.ndarray) -> float:
        """(beta / 2) sum_l <v_l, A v_l>_h."""
        return 0.5 * self.beta * self.inner(vl, sp.apply_A(vl, self.reg, self.d))


@dataclass
class State:
    """The outer iterate's cached forward solve (what every matvec reads)."""
    vl: np.ndarray
    traj: tr.Trajectory
    J: float
    J_dist: float
    J_reg: float
    g: Optional[np.ndarray] = None


def objective(P: Problem, vl: np.ndarray) -> Tuple[float, float, float]:
    """(J, J_dist, J_reg) at v; one forward solve."""
    m1 = tr.forward_only(P.mT, vl, P.nt)
    jd = 0.5 * P.hd * float(np.sum((P.mR - m1) ** 2))
    jr = P.reg_energy(vl)
    return jd + jr, jd, jr


def objective_gradient(P: Problem, vl: np.ndarray) -> State:
    """Forward solve, adjoint solve and reduced gradient g = beta A v + K[F]."""
    traj = tr.forward_state(P.mT, vl, P.nt)
    jd = 0.5 * P.hd * float(np.sum((P.mR - traj.m1) ** 2))
    jr = P.reg_energy(vl)
    _, F = tr.adjoint_with_force(P.mR - traj.m1, vl, traj, P.nt)
    g = P.beta * sp.apply_A(vl, P.reg, P.d) + P.project(F)
    return State(vl.copy(), traj, jd + jr, jd, jr, g)


def incremental_m1(P: Problem, S: State, vtl: np.ndarray) -> np.ndarray:
    """m~_1 of the incremental state equation at the cached iterate."""
    return tr.incremental_state(S.vl, vtl, S.traj, P.nt)


def hessian_matvec(P: Problem, S: State, vtl: np.ndarray) -> np.ndarray:
    """GN Hessian matvec H v~ = beta A v~ + K[F~] (Algorithm a:hessian-matvec)."""
    mt1 = tr.incremental_state(S.vl, vtl, S.traj, P.nt)
    _, Ft = tr.adjoint_with_force(-mt1, S.vl, S.traj, P.nt)
    return P.beta * sp.apply_A(vtl, P.reg, P.d) + P.project(Ft)


def newton_hessian_matvec(P: Problem, S: State, vtl: np.ndarray) -> np.ndarray:
    """Full-Newton Hessian matvec H v~ = beta A v~ + K[F~] with the lambda terms of
    e:sec-order-iadj and the incremental body force lam~ grad m + lam grad m~ kept
    (e:second-order-opt-cond); the Gauss-Newton matvec drops them."""
    mt1, gmt, gmts = tr.incremental_state_trajectory(S.vl, vtl, S.traj, P.nt)
    adj = tr.adjoint_trajectory(P.mR - S.traj.m1, S.vl, P.nt)
    Ft = tr.newton_adjoint_with_force(-mt1, S.vl, vtl, S.traj, adj, gmt, gmts, P.nt)
    return P.beta * sp.apply_A(vtl, P.reg, P.d) + P.project(Ft)


def precond(P: Problem, r: np.ndarray) -> np.ndarray:
    """(beta A)^-1 with the zero mode unscaled, per coefficient and component."""
    return sp.apply_Pinv(r, P.reg, P.beta, P.d)
