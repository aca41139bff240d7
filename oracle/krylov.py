"""PCG, Armijo line search and the Gauss-Newton outer iteration (FP64, CPU).

Paper: Section "Inexact Newton-Krylov Method" (PCG with the spectral
preconditioner, the inexact termination rule e:termination-criterion-ksm with
forcing eta_k = min(0.5, sqrt(||g_k|| / ||g_0||)), at most n inner iterations),
Algorithm a:outer-iteration, the Armijo backtracking line search of Section
"Numerical Optimization", the stopping rules e:stopping-criteria /
e:converged, the CFL guard of Section "Parameter Selection" (halve s_k until
the CFL condition holds, before the line search), and beta continuation
(divide beta by ten per level, warm start).

Readings where the paper is silent:
* PCG is the textbook preconditioned CG with x0 = 0 and Euclidean inner products
  (the h_d weight cancels in every ratio). It also stops on non-positive
  curvature <p, H p> <= 0.
* Armijo: alpha starts at 1, sufficient decrease J(v + a s) <= J(v) + c1 a <g, s>_h
  with c1 = 1e-4, alpha halved at most 20 times, then failure is reported.
* Convergence studies use ||g_k||_inf <= gtol * ||g_0||_inf ("relative change of
  the gradient of three orders", gtol = 1e-3), capped at max_outer iterations, or the
  paper's full rule ((C1 and C2 and C3) or C4 or C5) with tau_J (stopping_rule), where
  n_opt = max_outer and C5 reads k > n_opt literally (at most n_opt + 1 iterations).
* Continuation: a list of beta levels solved in turn, each warm-started from
  the previous level's solution, each with its own relative-gradient rule.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import reduced as rd
from .timebasis import velocity_at


def pcg(apply_H: Callable[[np.ndarray], np.ndarray],
        apply_Pinv: Callable[[np.ndarray], np.ndarray],
        rhs: np.ndarray, rtol: float, maxit: int) -> Tuple[np.ndarray, int, float, bool]:
    """Solve H x = rhs from x0 = 0; stop when ||r||_2 <= rtol ||rhs||_2.

    Non-positive curvature <p, H p> <= 0 ends the iteration (Section "GN
    Approximation": terminate the inner iteration on negative curvature). Reading:
    when that happens in the first iteration, x is the preconditioned residual
    direction p = P^-1 rhs (a descent direction) rather than zero, as in truncated
    Newton methods.

    Returns (x, iterations, ||r||/||rhs||, converged).
    """
    x = np.zeros_like(rhs)
    r = rhs.copy()
    nb = float(np.sqrt(np.sum(rhs * rhs)))
    if nb == 0.0:
        return x, 0, 0.0, True
    tol = rtol * nb
    z = apply_Pinv(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    it = 0
    rn = nb
    while it < maxit:
        if rn <= tol:
            return x, it, rn / nb, True
        Hp = apply_H(p)
        pHp = float(np.sum(p * Hp))
        if pHp <= 0.0:
            if it == 0:
                x = p.copy()
            break
        alpha = rz / pHp
        x = x + alpha * p
        r = r - alpha * Hp
        it += 1
        rn = float(np.sqrt(np.sum(r * r)))
        if rn <= tol:
            return x, it, rn / nb, True
        z = apply_Pinv(r)
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, rn / nb, rn <= tol


def cfl_number(vl: np.ndarray, nt: int) -> float:
    """h_t * max over t_j and i of ||v^i(t_j)||_inf / h_x^i (Section "Numerical Discretization")."""
    d = vl.shape[1]
    shape = vl.shape[2:]
    h = 1.0 / nt
    best = 0.0
    if vl.shape[0] == 1:
        times = [0.0]
    else:
        times = [j * h for j in range(nt + 1)]
    for t in times:
        v = velocity_at(vl, t)
        for i in range(d):
            hx = 2.0 * math.pi / shape[i]
            best = max(best, float(np.abs(v[i]).max()) / hx)
    return h * best


def armijo(P: rd.Problem, vl: np.ndarray, J: float, g: np.ndarray, s: np.ndarray,
           c1: float = 1e-4, max_halvings: int = 20) -> Tuple[float, bool, int]:
    """Backtracking from alpha = 1; returns (alpha, success, trial count). A trial whose
    transport overflows (non-finite J) is rejected like one that does not decrease J."""
    slope = P.inner(g, s)
    alpha = 1.0
    for trial in range(max_halvings + 1):
        with np.errstate(over="ignore", invalid="ignore"):
            Jt, _, _ = rd.objective(P, vl + alpha * s)
        if math.isfinite(Jt) and Jt <= J + c1 * alpha * slope:
            return alpha, True, trial + 1
        alpha *= 0.5
    return 0.0, False, max_halvings + 1


@dataclass
class SolveReport:
    iterations: int = 0
    cg_iterations: List[int] = field(default_factory=list)
    alphas: List[float] = field(default_factory=list)
    J: List[float] = field(default_factory=list)
    gnorm_inf: List[float] = field(default_factory=list)
    n_pde: int = 0
    matvecs: int = 0
    gnorm0_inf: float = 0.0
    converged: bool = False
    line_search_failed: bool = False
    reason: str = ""


def gauss_newton(P: rd.Problem, v0: Optional[np.ndarray] = None, gtol: float = 1e-3,
                 max_outer: int = 50, rule: str = "relgrad", tau_J: float = 1e-3,
                 cfl_max: Optional[float] = None, pcg_maxit: Optional[int] = None,
                 gref_inf: Optional[float] = None, hessian: str = "gn"
                 ) -> Tuple[np.ndarray, SolveReport, rd.State]:
    """Algorithm a:outer-iteration with GN-PCG search directions.

    gref_inf: gradient scale of the relative-gradient rule (default: this solve's
    ||g_0||_inf). A continuation passes its first level's value (see continuation).
    hessian: "gn" (e:gauss-newton) or "newton" (e:second-order-opt-cond)."""
    matvec = rd.newton_hessian_matvec if hessian == "newton" else rd.hessian_matvec
    vl = np.zeros(P.vshape()) if v0 is None else v0.copy()
    n = int(np.prod(P.vshape()))
    maxit = n if pcg_maxit is None else pcg_maxit
    rep = SolveReport()
    S = rd.objective_gradient(P, vl)
    rep.n_pde += 2
    J0 = S.J
    g0_2 = float(np.sqrt(np.sum(S.g * S.g)))
    g0_inf = float(np.abs(S.g).max()) if not gref_inf else float(gref_inf)
    rep.gnorm0_inf = float(np.abs(S.g).max())
    rep.J.append(S.J)
    rep.gnorm_inf.append(g0_inf)
    J_prev: Optional[float] = None
    v_prev: Optional[np.ndarray] = None
    k = 0
    while True:
        ginf = float(np.abs(S.g).max())
        if rule == "relgrad":
            if ginf <= gtol * g0_inf or g0_inf == 0.0:
                rep.converged, rep.reason = True, "relative gradient"
                break
            if k >= max_outer:
                rep.reason = "max outer iterations"
                break
        else:
            stop, crit = stopping_rule(k, J0, J_prev, S.J, v_prev, vl, S.g, tau_J, max_outer)
            if stop:
                rep.converged = bool(crit["C4"] or (crit["C1"] and crit["C2"] and crit["C3"]))
                rep.reason = "C1-C3" if crit["C1"] and crit["C2"] and crit["C3"] else ("C4" if crit["C4"] else "C5")
                break
        g2 = float(np.sqrt(np.sum(S.g * S.g)))
        eta = min(0.5, math.sqrt(g2 / g0_2))
        s, its, _, _ = pcg(lambda w: matvec(P, S, w), lambda r: rd.precond(P, r), -S.g, eta, maxit)
        rep.cg_iterations.append(its)
        rep.matvecs += its
        rep.n_pde += 2 * its
        if cfl_max is not None:
            while cfl_number(vl + s, P.nt) > cfl_max:
                s = 0.5 * s
        alpha, ok, trials = armijo(P, vl, S.J, S.g, s)
        rep.n_pde += trials
        if not ok:
            rep.line_search_failed, rep.reason = True, "line search failed"
            break
        rep.alphas.append(alpha)
        J_prev, v_prev = S.J, vl
        vl = vl + alpha * s
        S = rd.objective_gradient(P, vl)
        rep.n_pde += 2
        rep.J.append(S.J)
        rep.gnorm_inf.append(float(np.abs(S.g).max()))
        k += 1
    rep.iterations = k
    return vl, rep, S


def stopping_rule(k: int, J0: float, J_prev: Optional[float], J: float, v_prev: Optional[np.ndarray],
                  v: np.ndarray, g: np.ndarray, tau_J: float, n_opt: int,
                  eps_mach: float = float(np.finfo(np.float64).eps)) -> Tuple[bool, dict]:
    """Termination rule of the outer iteration, e:stopping-criteria combined as in
    e:converged: stop if (C1 and C2 and C3) or C4 or C5, with

      C1  J(v_{k-1}) - J(v_k)        < tau_J (1 + J(v_0))
      C2  ||v_{k-1} - v_k||_inf      < sqrt(tau_J) (1 + ||v_k||_inf)
      C3  ||g_k||_inf                < tau_J^(1/3) (1 + J(v_0))
      C4  ||g_k||_inf                < 1e3 eps_mach
      C5  k                          > n_opt

    evaluated at the top of the loop of Algorithm a:outer-iteration, k being the number
    of completed outer iterations. C1-C3 compare two iterates and are false at k = 0.
    eps_mach is FP64's for both transport precisions (the reductions are FP64).
    Returns (stop, {"C1": .., ..., "C5": ..})."""
    ginf = float(np.abs(g).max())
    crit = {"C1": False, "C2": False, "C3": False,
            "C4": ginf < 1e3 * eps_mach,
            "C5": k > n_opt}
    if k > 0:
        crit["C1"] = (J_prev - J) < tau_J * (1.0 + J0)
        crit["C2"] = float(np.abs(v_prev - v).max()) < math.sqrt(tau_J) * (1.0 + float(np.abs(v).max()))
        crit["C3"] = ginf < tau_J ** (1.0 / 3.0) * (1.0 + J0)
    stop = (crit["C1"] and crit["C2"] and crit["C3"]) or crit["C4"] or crit["C5"]
    return bool(stop), crit


def scale_memory(alpha_tilde: float, alpha: float) -> float:
    """Step-scale memory of the Picard scheme (Section "Parameter Selection",
    "Optimization"): the next direction is scaled by alpha~ before the line search;
    if the line search had to backtrack (alpha < 1), alpha~ shrinks by alpha,
    and if alpha = 1 was accepted, alpha~ doubles."""
    return alpha_tilde * alpha if alpha < 1.0 else 2.0 * alpha_tilde


def picard(P: rd.Problem, v0: Optional[np.ndarray] = None, gtol: float = 1e-3, max_outer: int = 500,
           memory: bool = True, stagnation: Tuple[int, float] = (10, 1e-6),
           gref_inf: Optional[float] = None) -> Tuple[np.ndarray, SolveReport, rd.State]:
    """Globalised Picard iteration (preconditioned gradient descent), e:picard.

    The Picard iterate -(beta A)^-1 [gamma grad p + f] is used as a search direction
    by subtracting the current iterate; with the eliminated pressure that is
    s_k = -P^-1 g_k, P = beta A with the zero mode unscaled (Section "Picard
    Method"). s_k is scaled by the memory alpha~ (scale_memory) and enters the
    Armijo line search from alpha = 1. Stops on the relative-gradient rule, after
    max_outer iterations, or when the objective changed by at most stagnation[1]
    (relative to 1 + J_0) in each of stagnation[0] consecutive iterations (the
    rule of Section "Convergence Study" for the Picard method).
    """
    vl = np.zeros(P.vshape()) if v0 is None else v0.copy()
    rep = SolveReport()
    S = rd.objective_gradient(P, vl)
    rep.n_pde += 2
    rep.gnorm0_inf = float(np.abs(S.g).max())
    g0 = rep.gnorm0_inf if not gref_inf else float(gref_inf)
    J0 = S.J
    rep.J.append(S.J)
    rep.gnorm_inf.append(rep.gnorm0_inf)
    at = 1.0
    flat = 0
    k = 0
    while True:
        ginf = float(np.abs(S.g).max())
        if ginf <= gtol * g0 or g0 == 0.0:
            rep.converged, rep.reason = True, "relative gradient"
            break
        if flat >= stagnation[0]:
            rep.converged, rep.reason = True, "objective stagnates"
            break
        if k >= max_outer:
            rep.reason = "max outer iterations"
            break
        s = -(at if memory else 1.0) * rd.precond(P, S.g)
        alpha, ok, trials = armijo(P, vl, S.J, S.g, s)
        rep.n_pde += trials
        if not ok:
            rep.line_search_failed, rep.reason = True, "line search failed"
            break
        rep.alphas.append(alpha)
        if memory:
            at = scale_memory(at, alpha)
        J_prev = S.J
        vl = vl + alpha * s
        S = rd.objective_gradient(P, vl)
        rep.n_pde += 2
        rep.J.append(S.J)
        rep.gnorm_inf.append(float(np.abs(S.g).max()))
        flat = flat + 1 if abs(J_prev - S.J) <= stagnation[1] * (1.0 + J0) else 0
        k += 1
    rep.iterations = k
    return vl, rep, S


def continuation(P: rd.Problem, betas: Sequence[float], gtol: float = 1e-3,
                 max_outer: int = 50, cfl_max: Optional[float] = None
                 ) -> Tuple[np.ndarray, List[SolveReport]]:
    """Solve for each beta in turn, warm-starting from the previous level.

    Reading: every level's relative-gradient rule is measured against the first
    level's ||g_0||_inf (a warm-started level's own g_0 is already small)."""
    vl = np.zeros(P.vshape())
    reports = []
    gref = None
    for b in betas:
        Pb = rd.Problem(P.mT, P.mR, P.nt, P.nc, P.reg, P.gamma, b)
        vl, rep, _ = gauss_newton(Pb, vl, gtol=gtol, max_outer=max_outer, cfl_max=cfl_max, gref_inf=gref)
        if gref is None:
            gref = rep.gnorm0_inf
        reports.append(rep)
    return vl, reports


@dataclass
class BetaTrial:
    beta: float
    min_det: float
    l2_rel: float
    accepted: bool


@dataclass
class BetaSearchReport:
    trials: List[BetaTrial] = field(default_factory=list)
    beta_star: float = float("nan")
    min_det_star: float = float("nan")
    l2_rel_star: float = float("nan")
    dbeta_min: float = 0.0
    breached: bool = False
    reason: str = ""

    @property
    def steps(self) -> int:
        return len(self.trials)


def beta_search_logic(evaluate: Callable[[float, Optional[np.ndarray]], Tuple[np.ndarray, float, float]],
                      eps_F: float, beta_start: float = 1.0, beta_min: float = 1e-6,
                      dbeta_rel: float = 0.05, l2_rel_min: float = 1e-2, max_steps: int = 64
                      ) -> Tuple[Optional[np.ndarray], BetaSearchReport]:
    """Parameter continuation in beta with a lower bound eps_F on det F_1.

    Section "Parameter Selection" (parameter continuation) and Table t:para-cont:
    solve at a large beta (underfitting), reduce beta by one order of magnitude
    while min det F_1 >= eps_F, then bisect between the last accepted and the
    breaching beta; stop when the change in beta drops below 5% of the beta at
    which eps_F was breached. beta is bounded below by 1e-6, and the descent
    also stops when the relative change of the L2 distance drops below 1e-2.

    evaluate(beta, v_warm) solves at beta (warm-started from v_warm, None = zero)
    and returns (v, min det F_1, ||m_R - m_1|| / ||m_R - m_T||).

    Readings: the bisection midpoint is the arithmetic mean; every trial is
    warm-started from the last accepted solution; the bisection step is half the
    bracket, and it stops once that is below dbeta_rel times the first breaching
    beta (these reproduce the steps, beta* and dbeta_min of Table t:para-cont).
    """
    rep = BetaSearchReport()
    v_ok: Optional[np.ndarray] = None
    beta_ok: Optional[float] = None
    det_ok = l2_ok = float("nan")

    def trial(beta: float):
        v, d, l2 = evaluate(beta, v_ok)
        acc = d >= eps_F
        rep.trials.append(BetaTrial(beta, d, l2, acc))
        return v, d, l2, acc

    beta = beta_start
    breach: Optional[float] = None
    while True:
        v, d, l2, acc = trial(beta)
        if not acc:
            breach = beta
            break
        prev_l2 = l2_ok if beta_ok is not None else None
        v_ok, beta_ok, det_ok, l2_ok = v, beta, d, l2
        if rep.steps >= max_steps:
            rep.reason = "step limit"
            break
        if prev_l2 is not None and abs(prev_l2 - l2) < l2_rel_min * prev_l2:
            rep.reason = "L2 distance stagnates"
            break
        if beta / 10.0 < beta_min:
            rep.reason = "lower bound on beta"
            break
        beta = beta / 10.0
    if breach is not None:
        rep.breached = True
        if beta_ok is None:
            rep.reason = "bound breached at the first beta"
            return None, rep
        lo, hi = breach, beta_ok
        rep.dbeta_min = dbeta_rel * breach
        rep.reason = "bisection converged"
        while (hi - lo) / 2.0 >= rep.dbeta_min:
            if rep.steps >= max_steps:
                rep.reason = "step limit"
                break
            mid = (lo + hi) / 2.0
            v, d, l2, acc = trial(mid)
            if acc:
                v_ok, beta_ok, det_ok, l2_ok = v, mid, d, l2
                hi = mid
            else:
                lo = mid
    rep.beta_star, rep.min_det_star, rep.l2_rel_star = beta_ok, det_ok, l2_ok
    return v_ok, rep


def beta_search(P: rd.Problem, eps_F: float, beta_start: float = 1.0, gtol: float = 1e-3,
                max_outer: int = 50, **kw) -> Tuple[Optional[np.ndarray], BetaSearchReport]:
    """beta_search_logic with GN-PCG solves (relative-gradient rule against the first
    solve's ||g_0||_inf) and det F_1 from the deformation-gradient solve."""
    from . import defgrad as dg
    r0 = float(np.sqrt(np.sum((P.mR - P.mT) ** 2)))
    gref: List[Optional[float]] = [None]

    def evaluate(beta: float, v_warm: Optional[np.ndarray]):
        Pb = rd.Problem(P.mT, P.mR, P.nt, P.nc, P.reg, P.gamma, beta)
        v, rep, S = gauss_newton(Pb, v_warm, gtol=gtol, max_outer=max_outer, gref_inf=gref[0])
        if gref[0] is None:
            gref[0] = rep.gnorm0_inf
        _, stats = dg.det_stats(v, P.nt)
        return v, stats[0], math.sqrt(2.0 * S.J_dist / P.hd) / r0

    return beta_search_logic(evaluate, eps_F, beta_start, **kw)
