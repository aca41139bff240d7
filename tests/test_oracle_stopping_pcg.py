"""Pins of the oracle's termination rule (e:stopping-criteria, e:converged) and of PCG's
exit on non-positive curvature (Section "GN Approximation").

The termination rule is pinned with hand-built values, chosen so that each plausible
slip fails a test: sqrt(tau_J) against tau_J^(1/3) in C2 and C3, 1 + J(v_0) against
1 + J(v_k) in C1 and C3, ||v_k|| in C2, 1e3 eps_mach in C4, and k > n_opt in C5.
PCG's curvature exits are pinned on small indefinite matrices with an SPD
preconditioner, against numpy's dense solve and the one-step closed form.
"""
import math

import numpy as np
import pytest

from oracle import krylov as kr
from oracle import reduced as rd
from oracle import transport as tr
import synth

TAU = 1e-3            # sqrt = 0.0316..., cube root = 0.1
EPS = float(np.finfo(np.float64).eps)


def rule(k, J0=9.0, J_prev=3.0, J=2.995, dv=0.01, vmax=1.0, gmax=0.5, n_opt=50):
    v = np.full((1, 2, 4, 4), vmax)
    v_prev = v + dv
    g = np.zeros((1, 2, 4, 4))
    g[0, 1, 2, 3] = -gmax
    return kr.stopping_rule(k, J0, J_prev, J, v_prev, v, g, TAU, n_opt)


def test_c1_scales_the_decrease_by_the_initial_objective():
    # threshold tau (1 + J0) = 1e-2; with 1 + J_k = 3.995 it would be 4.0e-3
    assert rule(1, J_prev=3.0, J=2.995)[1]["C1"]
    assert not rule(1, J_prev=3.0, J=2.989)[1]["C1"]
    # an increase of J also satisfies C1 (the decrease is negative)
    assert rule(1, J_prev=3.0, J=3.5)[1]["C1"]


def test_c2_uses_the_square_root_of_tau_and_the_new_iterate():
    # threshold sqrt(tau) (1 + ||v_k||) = 0.0632 for ||v_k|| = 1; the cube root would give 0.2
    assert rule(1, dv=0.05)[1]["C2"]
    assert not rule(1, dv=0.1)[1]["C2"]
    # ||v_k|| = 3: threshold 0.126
    assert rule(1, dv=0.1, vmax=3.0)[1]["C2"]


def test_c3_uses_the_cube_root_of_tau_and_the_initial_objective():
    # threshold tau^(1/3) (1 + J0) = 1.0; sqrt(tau) would give 0.316, 1 + J_k 0.3995
    assert rule(1, gmax=0.5)[1]["C3"]
    assert not rule(1, gmax=1.01)[1]["C3"]
    assert rule(1, J0=0.0, gmax=0.09)[1]["C3"] and not rule(1, J0=0.0, gmax=0.11)[1]["C3"]


def test_c1_to_c3_compare_two_iterates_and_are_false_at_the_start():
    stop, crit = rule(0)
    assert not stop and not (crit["C1"] or crit["C2"] or crit["C3"])


def test_c4_machine_precision_gradient_and_c5_iteration_budget():
    assert 1e3 * EPS == pytest.approx(2.220446049250313e-13)
    stop, crit = rule(0, gmax=2.0e-13)
    assert stop and crit["C4"] and not crit["C5"]
    stop, crit = rule(0, gmax=2.5e-13)
    assert not stop and not crit["C4"]
    # C5 reads k > n_opt: the iterate index n_opt still continues, n_opt + 1 stops
    assert not rule(5, J=1.0, n_opt=5)[0]
    stop, crit = rule(6, J=1.0, n_opt=5)
    assert stop and crit["C5"] and not crit["C1"]


def test_conjunction_first_holds_at_a_known_iteration():
    """A hand-built run: (J_k, ||v_{k-1} - v_k||, ||g_k||) for k = 0..4. C1 fails at k = 1
    (large decrease), C2 at k = 2 (large step), C3 at k = 3 (large gradient); all three
    hold first at k = 4, and only the conjunction (not any one criterion) stops there."""
    J = [9.0, 4.0, 3.999, 3.998, 3.997]
    dv = [None, 0.01, 0.5, 0.01, 0.01]
    g = [5.0, 0.5, 0.5, 1.5, 0.5]
    stops = []
    for k in range(5):
        stop, crit = rule(k, J0=J[0], J_prev=J[k - 1] if k else None, J=J[k], dv=dv[k] or 0.0, gmax=g[k])
        stops.append(stop)
        if k == 1:
            assert not crit["C1"] and crit["C2"] and crit["C3"]
        if k == 2:
            assert crit["C1"] and not crit["C2"] and crit["C3"]
        if k == 3:
            assert crit["C1"] and crit["C2"] and not crit["C3"]
    assert stops == [False, False, False, False, True]


def small_problem(shape=(16, 16), nt=8, reg=2, beta=1e-1):
    mT = synth.smooth_image(shape, 5, 8.0)
    vstar = synth.bandlimited_velocity(shape, 77, 3, 0.8)
    mR = tr.forward_only(mT, vstar, nt)
    return rd.Problem(mT, mR, nt, 1, reg, 0, beta)


def test_gauss_newton_with_the_paper_rule_honours_c5_literally():
    """With a tolerance no solve meets, the paper's rule stops by C5 after n_opt + 1
    iterations and reports no convergence."""
    P = small_problem()
    for n_opt in (0, 2):
        _, rep, _ = kr.gauss_newton(P, gtol=0.0, rule="paper", tau_J=1e-30, max_outer=n_opt)
        assert rep.iterations == n_opt + 1 and not rep.converged and rep.reason == "C5"


def test_gauss_newton_with_the_paper_rule_stops_on_the_conjunction():
    """At tau_J = 1e-3 the solve stops on C1-C3, and C1 and C3 hold when re-evaluated
    from the run's own record of J and ||g||_inf."""
    P = small_problem()
    v, rep, S = kr.gauss_newton(P, gtol=0.0, rule="paper", tau_J=TAU, max_outer=50)
    assert rep.converged and rep.reason == "C1-C3"
    k = rep.iterations
    J = rep.J
    assert k >= 1
    assert (J[k - 1] - J[k]) < TAU * (1 + J[0])
    assert rep.gnorm_inf[k] < TAU ** (1 / 3) * (1 + J[0])


def orthogonal(n, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return q


def test_pcg_negative_curvature_in_the_first_step_returns_the_preconditioned_rhs():
    """Reading of the curvature exit in the first iteration: x = P^-1 rhs (a descent
    direction) with 0 iterations. H has eigenvalues (-1, 2, 3, 5) in a rotated basis; P is
    SPD; rhs = P u for the eigenvector u of -1, so the first direction P^-1 rhs = u has
    curvature u.H.u = -1."""
    Q = orthogonal(4, 3)
    H = Q @ np.diag([-1.0, 2.0, 3.0, 5.0]) @ Q.T
    B = np.random.default_rng(4).standard_normal((4, 4))
    Pm = B @ B.T + 4 * np.eye(4)
    u = Q[:, 0]
    rhs = Pm @ u
    x, its, relres, ok = kr.pcg(lambda w: H @ w, lambda r: np.linalg.solve(Pm, r), rhs, 1e-12, 4)
    assert its == 0 and not ok
    assert np.abs(x - np.linalg.solve(Pm, rhs)).max() < 1e-14
    assert np.abs(x - u).max() < 1e-12
    assert relres == 1.0


def test_pcg_negative_curvature_after_the_first_step_keeps_the_iterate():
    """H = diag(2, -1), P = I, rhs = (1, 0.9): the first direction has curvature
    2 - 0.81 > 0, the second is negative; PCG stops after one update, x = (r.r / r.H.r) r."""
    H = np.diag([2.0, -1.0])
    rhs = np.array([1.0, 0.9])
    x, its, relres, ok = kr.pcg(lambda w: H @ w, lambda r: r, rhs, 1e-12, 10)
    a0 = rhs @ rhs / (rhs @ H @ rhs)
    x1 = a0 * rhs
    r1 = rhs - a0 * (H @ rhs)
    p1 = r1 + (r1 @ r1) / (rhs @ rhs) * rhs
    assert p1 @ H @ p1 <= 0.0
    assert its == 1 and not ok
    assert np.abs(x - x1).max() < 1e-15
    assert relres == pytest.approx(math.sqrt(r1 @ r1) / math.sqrt(rhs @ rhs), rel=1e-14)
