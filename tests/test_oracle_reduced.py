"""Pins of the oracle's objective, reduced gradient and GN Hessian matvec.

Taylor tests (finite differences of J against <g, w>_h), closed forms at v = 0,
the zero-residual identities, Hessian symmetry and energy, and the extremes of
the paper's Table t:eigenvalues.
"""
import json
import os

import numpy as np
import pytest

from oracle import reduced as rd
from oracle import spectral as sp
from oracle import transport as tr
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def make_problem(shape=(16, 16), nt=6, nc=1, reg=1, gamma=0, beta=1e-2, zero_residual=False):
    mT = synth.smooth_image(shape, 5, 8.0)
    vstar = synth.bandlimited_velocity(shape, 77, 3, 0.8, divfree=bool(gamma), nc=nc)
    if zero_residual:
        mR = tr.forward_only(mT, vstar, nt)
    else:
        mR = synth.smooth_image(shape, 6, 8.0)
    return rd.Problem(mT, mR, nt, nc, reg, gamma, beta), vstar


def direction(shape, nc, seed, divfree):
    return synth.bandlimited_velocity(shape, seed, 4, 0.3, divfree=divfree, nc=nc)


@pytest.mark.parametrize("nc,reg,gamma", [(1, 1, 0), (2, 2, 0), (3, 2, 1), (1, 1, 1)])
def test_gradient_taylor(nc, reg, gamma):
    P, vstar = make_problem(nc=nc, reg=reg, gamma=gamma)
    v = 0.7 * vstar
    w = direction(P.shape, nc, 91, bool(gamma))
    S = rd.objective_gradient(P, v)
    gw = P.inner(S.g, w)
    errs = []
    for eps in (1e-2, 1e-3, 1e-4):
        fd = (rd.objective(P, v + eps * w)[0] - rd.objective(P, v - eps * w)[0]) / (2 * eps)
        errs.append(abs(fd - gw) / abs(gw))
    assert errs[2] < 1e-8, errs
    assert errs[0] / errs[1] > 30, errs


def test_gradient_at_zero_velocity_closed_form():
    P, _ = make_problem(nc=1, reg=2, gamma=1)
    S = rd.objective_gradient(P, np.zeros(P.vshape()))
    ref = sp.apply_K((P.mR - P.mT) * sp.grad(P.mT))
    assert np.abs(S.g[0] - ref).max() < 1e-14 * 10 * np.abs(ref).max() + 1e-16


def test_gradient_at_zero_velocity_nonstationary_uses_heun_weights():
    # v = 0: the body force is constant in time, so g_l = (sum_j h/2 (b_l(t_j) + b_l(t_j+1))) f.
    P, _ = make_problem(nc=3, reg=1, gamma=0)
    S = rd.objective_gradient(P, np.zeros(P.vshape()))
    f = (P.mR - P.mT) * sp.grad(P.mT)
    h = 1.0 / P.nt
    t = np.arange(P.nt + 1) * h
    cheb = [np.ones_like(t), 2 * t - 1, 2 * (2 * t - 1) ** 2 - 1]
    for l in range(3):
        wl = np.sum(0.5 * h * (cheb[l][:-1] + cheb[l][1:]))
        assert np.abs(S.g[l] - wl * f).max() < 1e-13


def test_gradient_at_true_velocity_is_the_regulariser():
    P, vstar = make_problem(nc=2, reg=2, gamma=0, zero_residual=True)
    S = rd.objective_gradient(P, vstar)
    ref = P.beta * sp.apply_A(vstar, P.reg, P.d)
    assert S.J_dist < 1e-28
    assert np.abs(S.g - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("nc,reg,gamma", [(1, 1, 0), (2, 2, 0), (2, 2, 1)])
def test_hessian_symmetry_and_energy(nc, reg, gamma):
    P, vstar = make_problem(nc=nc, reg=reg, gamma=gamma)
    S = rd.objective_gradient(P, 0.6 * vstar)
    u = direction(P.shape, nc, 101, bool(gamma))
    w = direction(P.shape, nc, 102, bool(gamma))
    Hu = rd.hessian_matvec(P, S, u)
    Hw = rd.hessian_matvec(P, S, w)
    a, b = P.inner(u, Hw), P.inner(Hu, w)
    assert abs(a - b) <= 1e-13 * abs(a)
    mt = rd.incremental_m1(P, S, w)
    energy = P.beta * P.inner(w, sp.apply_A(w, reg, 2)) + P.inner(mt, mt)
    assert abs(P.inner(w, Hw) - energy) <= 1e-13 * energy


@pytest.mark.parametrize("nc", [1, 2])
def test_zero_residual_gradient_derivative_equals_gn_matvec(nc):
    """At m_R = m_1(v*), lambda = 0, so GN equals full Newton: dg/dv [w] = H w."""
    P, vstar = make_problem(nc=nc, reg=1, gamma=0, zero_residual=True)
    S = rd.objective_gradient(P, vstar)
    w = direction(P.shape, nc, 103, False)
    Hw = rd.hessian_matvec(P, S, w)
    eps = 1e-4
    gp = rd.objective_gradient(P, vstar + eps * w).g
    gm = rd.objective_gradient(P, vstar - eps * w).g
    fd = (gp - gm) / (2 * eps)
    assert np.abs(fd - Hw).max() <= 1e-8 * np.abs(Hw).max()


def test_hessian_at_zero_velocity_closed_form():
    """v = 0: H w = beta A w + K[(w . grad m_T) grad m_T] (linearised optical flow)."""
    P, _ = make_problem(nc=1, reg=2, gamma=1)
    S = rd.objective_gradient(P, np.zeros(P.vshape()))
    w = direction(P.shape, 1, 104, True)
    Hw = rd.hessian_matvec(P, S, w)
    gm = sp.grad(P.mT)
    ref = P.beta * sp.apply_A(w, 2, 2)[0] + sp.apply_K(np.sum(w[0] * gm, axis=0) * gm)
    assert np.abs(Hw[0] - ref).max() < 1e-12 * np.abs(ref).max()


def dense_hessian(P, S):
    n = int(np.prod(P.vshape()))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(rd.hessian_matvec(P, S, e.reshape(P.vshape())).reshape(-1))
    return np.stack(cols, axis=1)


def test_stokes_hessian_spectrum_contains_beta_a_on_curl_free_modes():
    """Table t:eigenvalues (Stokes): K reaches only the body force, so with respect to
    gradients (+) divergence-free fields H is block lower-triangular: the gradient part of
    H grad(phi_k) is beta * a(k) grad(phi_k), every beta * a(k) is an eigenvalue, and the
    smallest eigenvalue is beta (|k| = 1)."""
    P, vstar = make_problem(shape=(8, 8), nt=4, nc=1, reg=1, gamma=1, beta=1e-3)
    P.mT = synth.smooth_image((8, 8), 5, 8.0) * 8.0  # strong image gradients
    P.mR = synth.smooth_image((8, 8), 6, 8.0) * 8.0
    S = rd.objective_gradient(P, 0.5 * vstar)
    H = dense_hessian(P, S)
    ev = np.sort(np.linalg.eigvals(H).real)
    x1, x2 = synth.grid_coords((8, 8))
    for (k1, k2) in [(1, 0), (0, 1), (1, 2), (3, 1)]:
        w = np.stack([-k1 * np.sin(k1 * x1 + k2 * x2), -k2 * np.sin(k1 * x1 + k2 * x2)])[None]
        Hw = rd.hessian_matvec(P, S, w)
        lam = P.beta * (k1 * k1 + k2 * k2)
        grad_part = Hw[0] - sp.apply_K(Hw[0])
        assert np.abs(grad_part - lam * w[0]).max() < 1e-12 * np.abs(Hw).max()
        assert np.min(np.abs(ev - lam)) < 1e-10
    with open(os.path.join(GOLDEN, "eigen_extremes.json")) as fh:
        gold = [e for e in json.load(fh)["entries"] if "min_real" in e][0]
    assert gold["beta"] == P.beta
    assert ev[0] == pytest.approx(gold["min_real"], rel=1e-9)


@pytest.mark.parametrize("reg,gamma,key", [(2, 0, "H2"), (1, 1, "Stokes")])
def test_hessian_rayleigh_quotient_at_corner_mode_matches_paper(reg, gamma, key):
    """Table t:eigenvalues, beta = 1e6 on 64^2: the largest eigenvalue is the regulariser's
    corner symbol; the data term is negligible at that beta."""
    with open(os.path.join(GOLDEN, "eigen_extremes.json")) as fh:
        table = json.load(fh)
    gold = [e for e in table["entries"] if e["scheme"] == key and "max_real" in e][0]
    shape = tuple(table["grid"])
    mT = synth.smooth_image(shape, 5, 36.0)
    mR = synth.smooth_image(shape, 6, 36.0)
    P = rd.Problem(mT, mR, 4, 1, reg, gamma, gold["beta"])
    S = rd.objective_gradient(P, np.zeros(P.vshape()))
    j1, j2 = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    corner = (-1.0) ** (j1 + j2)
    w = np.stack([corner, 0.0 * corner])[None]
    rq = P.inner(w, rd.hessian_matvec(P, S, w)) / P.inner(w, w)
    assert rq == pytest.approx(gold["max_real"], rel=5e-7)


@pytest.mark.parametrize("nc,reg,gamma", [(1, 1, 0), (2, 2, 0), (1, 2, 1)])
def test_newton_matvec_is_the_derivative_of_the_gradient_at_nonzero_residual(nc, reg, gamma):
    """Full-Newton matvec (e:second-order-opt-cond) against central differences of the
    exact discrete gradient at a point with a nonzero residual (lambda != 0): the error
    decays as eps^2 and reaches rounding level; the GN matvec misses the lambda terms."""
    P, vstar = make_problem(nc=nc, reg=reg, gamma=gamma)
    v = 0.6 * vstar
    S = rd.objective_gradient(P, v)
    w = direction(P.shape, nc, 105, bool(gamma))
    Hw = rd.newton_hessian_matvec(P, S, w)
    errs = []
    for eps in (1e-2, 1e-3, 1e-4):
        fd = (rd.objective_gradient(P, v + eps * w).g - rd.objective_gradient(P, v - eps * w).g) / (2 * eps)
        errs.append(np.abs(fd - Hw).max() / np.abs(Hw).max())
    assert errs[0] / errs[1] > 50 and errs[2] < 1e-8, errs
    gn = rd.hessian_matvec(P, S, w)
    assert np.abs(gn - Hw).max() > 1e3 * errs[2] * np.abs(Hw).max()


@pytest.mark.parametrize("nc,reg,gamma", [(1, 1, 0), (3, 2, 1)])
def test_newton_matvec_is_symmetric(nc, reg, gamma):
    P, vstar = make_problem(nc=nc, reg=reg, gamma=gamma)
    S = rd.objective_gradient(P, 0.6 * vstar)
    u = direction(P.shape, nc, 106, bool(gamma))
    w = direction(P.shape, nc, 107, bool(gamma))
    a = P.inner(u, rd.newton_hessian_matvec(P, S, w))
    b = P.inner(rd.newton_hessian_matvec(P, S, u), w)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_newton_matvec_equals_gn_at_zero_residual():
    """lambda = m_R - m_1 vanishes at the true velocity, and with it every term that
    separates the full-Newton from the Gauss-Newton matvec."""
    P, vstar = make_problem(nc=1, reg=1, gamma=0, zero_residual=True)
    S = rd.objective_gradient(P, vstar)
    w = direction(P.shape, 1, 108, False)
    Hn, Hg = rd.newton_hessian_matvec(P, S, w), rd.hessian_matvec(P, S, w)
    assert np.abs(Hn - Hg).max() <= 1e-10 * np.abs(Hg).max()
