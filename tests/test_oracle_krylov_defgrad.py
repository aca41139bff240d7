"""Pins of the oracle's PCG, line search, GN driver and deformation gradient."""
import numpy as np
import pytest

from oracle import defgrad as dg
from oracle import krylov as kr
from oracle import reduced as rd
from oracle import spectral as sp
from oracle import transport as tr
import synth


def small_problem(shape=(8, 8), nt=4, nc=1, reg=1, gamma=0, beta=1e-2):
    mT = synth.smooth_image(shape, 5, 8.0)
    vstar = synth.bandlimited_velocity(shape, 77, 3, 0.8, divfree=bool(gamma), nc=nc)
    mR = tr.forward_only(mT, vstar, nt)
    return rd.Problem(mT, mR, nt, nc, reg, gamma, beta), vstar


@pytest.mark.parametrize("reg", [1, 2])
def test_pcg_matches_dense_solve(reg):
    P, vstar = small_problem(reg=reg)
    S = rd.objective_gradient(P, 0.5 * vstar)
    n = int(np.prod(P.vshape()))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(rd.hessian_matvec(P, S, e.reshape(P.vshape())).reshape(-1))
    H = np.stack(cols, axis=1)
    assert np.all(np.linalg.eigvalsh(0.5 * (H + H.T)) > 0)
    rhs = -S.g
    x_ref = np.linalg.solve(H, rhs.reshape(-1)).reshape(P.vshape())
    x, its, relres, ok = kr.pcg(lambda w: rd.hessian_matvec(P, S, w), lambda r: rd.precond(P, r),
                                rhs, 1e-12, n)
    assert ok and its <= n
    assert np.abs(x - x_ref).max() <= 1e-9 * np.abs(x_ref).max()


def test_pcg_identity_preconditioner_on_spd_matrix_converges_in_n_steps():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((12, 12))
    H = B @ B.T + 12 * np.eye(12)
    b = rng.standard_normal(12)
    x, its, relres, ok = kr.pcg(lambda w: H @ w, lambda r: r, b, 1e-13, 12)
    assert ok and its <= 12
    assert np.abs(H @ x - b).max() < 1e-10


def test_pcg_zero_rhs_and_forcing_stop():
    H = np.diag(np.arange(1.0, 11.0))
    x, its, relres, ok = kr.pcg(lambda w: H @ w, lambda r: r, np.zeros(10), 0.5, 10)
    assert its == 0 and ok and not x.any()
    x, its, relres, ok = kr.pcg(lambda w: H @ w, lambda r: r, np.ones(10), 0.5, 10)
    assert ok and relres <= 0.5 and its < 10


def test_armijo_rejects_ascent_direction():
    P, vstar = small_problem()
    v = np.zeros(P.vshape())
    S = rd.objective_gradient(P, v)
    alpha, ok, trials = kr.armijo(P, v, S.J, S.g, S.g.copy())
    assert not ok and alpha == 0.0 and trials == 21


def test_gauss_newton_converges_with_full_steps():
    """GN-PCG rows of the paper's convergence tables: a handful of outer iterations
    (4 to 13 there) with every full step accepted."""
    P, vstar = small_problem(shape=(16, 16), nt=8, reg=2, beta=1e-1)
    v, rep, S = kr.gauss_newton(P, gtol=1e-3, max_outer=20)
    assert rep.converged
    assert rep.iterations <= 10
    assert all(a == 1.0 for a in rep.alphas)
    assert rep.J[-1] < rep.J[0]


def test_gauss_newton_reduces_mismatch_and_counts_pde_solves():
    P, vstar = small_problem(shape=(16, 16), nt=8, reg=1, beta=1e-3)
    v, rep, S = kr.gauss_newton(P, gtol=1e-3, max_outer=20)
    assert rep.converged
    mis0 = np.sum((P.mR - P.mT) ** 2)
    assert S.J_dist / (0.5 * P.hd * mis0) < 0.05
    # 2 PDE solves per gradient, 2 per matvec, 1 per line-search trial (one trial per
    # iteration when every full step is accepted)
    assert all(a == 1.0 for a in rep.alphas)
    assert rep.n_pde == 2 * (rep.iterations + 1) + 2 * rep.matvecs + rep.iterations


def test_stokes_driver_keeps_velocity_divergence_free():
    P, vstar = small_problem(shape=(16, 16), nt=8, reg=2, gamma=1, beta=1e-2)
    v, rep, S = kr.gauss_newton(P, gtol=1e-3, max_outer=10)
    assert rep.converged
    assert np.abs(sp.div(v[0])).max() < 1e-10 * max(1.0, np.abs(v).max())


def test_cfl_guard_halves_steps():
    v = np.zeros((1, 2, 16, 16))
    v[0, 0] = 1.0
    assert kr.cfl_number(v, 16) == pytest.approx(16 / (2 * np.pi) / 16)


def test_continuation_warm_starts():
    P, _ = small_problem(shape=(16, 16), nt=8, reg=2, beta=1e-3)
    v, reps = kr.continuation(P, [1e-1, 1e-2, 1e-3])
    assert len(reps) == 3 and all(r.converged for r in reps)


def test_continuation_measures_every_level_against_the_first_gradient():
    """Reading of the continuation's stopping rule: a warm-started level stops when its
    gradient falls below gtol times the first level's ||g_0||_inf."""
    P, _ = small_problem(shape=(16, 16), nt=8, reg=2, beta=1e-3)
    v, reps = kr.continuation(P, [1e-1, 1e-2])
    g0 = reps[0].gnorm0_inf
    assert reps[1].gnorm0_inf < g0
    assert reps[1].gnorm_inf[-1] <= 1e-3 * g0
    # a level that starts converged against that scale takes no step
    v2, reps2 = kr.continuation(P, [1e-1, 1e-1])
    assert reps2[1].iterations == 0


GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "beta_search_table.json")


@pytest.mark.parametrize("row,beta_c", [(0, 0.31), (1, 0.021), (2, 0.0335), (3, 2.65e-4)])
def test_beta_search_reproduces_table_para_cont(row, beta_c):
    """The search's control flow against Table t:para-cont: with a monotone det F_1(beta)
    that crosses eps_F at beta_c (any value between the last rejected and the accepted
    trial of that row), the steps, beta* and dbeta_min are the table's."""
    import json
    r = json.load(open(GOLDEN))["rows"][row]
    eps = r["eps_F"]

    def evaluate(beta, v_warm):
        return np.array([beta]), eps * beta / beta_c, 1.0 / (1.0 + np.log10(1.0 / beta))

    v, rep = kr.beta_search_logic(evaluate, eps)
    assert rep.steps == r["steps"], [t.beta for t in rep.trials]
    assert abs(rep.beta_star - r["beta_star"]) <= 1e-12 * r["beta_star"]
    assert abs(rep.dbeta_min - r["dbeta_min"]) <= 1e-12 * r["dbeta_min"]
    assert rep.breached and rep.min_det_star >= eps
    assert v[0] == rep.beta_star


def test_beta_search_warm_starts_from_the_last_accepted_solution_and_honours_bounds():
    calls = []

    def evaluate(beta, v_warm):
        calls.append((beta, None if v_warm is None else float(v_warm[0])))
        return np.array([beta]), 1.0, 0.5   # never breaches, L2 distance flat

    _, rep = kr.beta_search_logic(evaluate, 0.5)
    assert [c[0] for c in calls] == [1.0, 0.1]          # L2 distance stagnates after one decade
    assert calls[1][1] == 1.0 and rep.reason.startswith("L2")
    _, rep = kr.beta_search_logic(lambda b, w: (np.array([b]), 1.0, b), 0.5)
    assert rep.trials[-1].beta >= 1e-6 and rep.reason == "lower bound on beta"
    assert not rep.breached and rep.beta_star == rep.trials[-1].beta
    _, rep = kr.beta_search_logic(lambda b, w: (np.array([b]), 0.0, b), 0.5)
    assert rep.breached and rep.steps == 1 and np.isnan(rep.beta_star)


def test_beta_search_on_a_registration_problem():
    """Real solves: min det F_1 falls as beta falls; accepted trials satisfy the bound,
    rejected ones break it, and beta* lies within dbeta_min of a rejected beta."""
    shape, nt = (16, 16), 8
    mT = synth.smooth_image(shape, 3, 0.6 * 16 ** 2 / 16)
    vstar = synth.bandlimited_velocity(shape, 77, 2, 0.5, norm="linf")
    P = rd.Problem(mT, tr.forward_only(mT, vstar, nt), nt, 1, 1, 0, 1.0)
    v, rep = kr.beta_search(P, 0.8, max_outer=10)
    assert rep.breached and rep.reason == "bisection converged"
    for t in rep.trials:
        assert (t.min_det >= 0.8) == t.accepted
    acc = sorted((t.beta, t.min_det) for t in rep.trials)
    assert all(a[1] <= b[1] + 1e-9 for a, b in zip(acc, acc[1:]))   # det F_1 grows with beta
    rejected = [t.beta for t in rep.trials if not t.accepted]
    assert min(abs(rep.beta_star - b) for b in rejected) < 2 * rep.dbeta_min
    _, st = dg.det_stats(v, nt)
    assert st[0] == rep.min_det_star


def test_deformation_gradient_constant_velocity_is_identity():
    v = np.zeros((1, 2, 16, 16))
    v[0, 0], v[0, 1] = 0.4, -0.9
    F = dg.deformation_gradient(v, 6)
    assert np.abs(F[0, 0] - 1).max() < 1e-14 and np.abs(F[1, 1] - 1).max() < 1e-14
    assert np.abs(F[0, 1]).max() < 1e-14 and np.abs(F[1, 0]).max() < 1e-14


@pytest.mark.parametrize("shape", [(32, 32), (16, 16, 16)])
def test_det_divergence_free_is_one_to_second_order(shape):
    v = synth.bandlimited_velocity(shape, 12, 3, 0.8, divfree=True)
    errs = []
    for nt in (8, 16):
        _, (mn, mx, mean, std) = dg.det_stats(v, nt)
        errs.append(max(abs(mn - 1), abs(mx - 1)))
    assert errs[1] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_det_compressible_matches_jacobi_transport():
    """d/dt J + v . grad J = (div v) J with J(0) = 1 (Jacobi's formula), Heun in time."""
    shape = (32, 32)
    v = synth.c0_velocity(shape, 0.6)
    vv = v[0]
    dv = sp.div(vv)
    res = []
    for nt in (16, 32):
        h = 1.0 / nt
        J = np.ones(shape)
        for _ in range(nt):
            r1 = -np.sum(vv * sp.grad(J), axis=0) + dv * J
            Js = J + h * r1
            r2 = -np.sum(vv * sp.grad(Js), axis=0) + dv * Js
            J = J + 0.5 * h * (r1 + r2)
        det1, _ = dg.det_stats(v, nt)
        res.append(np.abs(det1 - J).max())
    assert res[1] < 1e-3 and res[0] / res[1] > 3.0


def test_picard_step_memory_follows_the_paper():
    """alpha~ shrinks by alpha when the line search backtracks and doubles when alpha = 1."""
    assert kr.scale_memory(1.0, 1.0) == 2.0
    assert kr.scale_memory(4.0, 0.25) == 1.0
    assert kr.scale_memory(0.5, 0.5) == 0.25


def test_picard_first_direction_is_the_picard_iterate_minus_v():
    """e:picard: the direction is -(beta A)^-1 [K f] - v on every nonzero mode (the
    Picard iterate minus the current iterate); the zero mode is left unscaled."""
    P, vstar = small_problem(shape=(16, 16), nt=6, reg=2, gamma=1, beta=1e-2)
    v = 0.4 * vstar
    S = rd.objective_gradient(P, v)
    f = S.g - P.beta * sp.apply_A(v, P.reg, P.d)          # K[f] (the projected body force)
    s = -rd.precond(P, S.g)
    kx = np.fft.fftfreq(16, 1.0 / 16)
    a = (kx[:, None] ** 2 + kx[None, :] ** 2) ** 2        # |k|^4 for H2
    for c in range(2):
        F = np.fft.fft2(f[0, c])
        V = np.fft.fft2(v[0, c])
        Sh = np.fft.fft2(s[0, c])
        nz = a > 0
        assert np.abs(Sh[nz] - (-F[nz] / (P.beta * a[nz]) - V[nz])).max() <= 1e-10 * np.abs(Sh).max()


def test_picard_reaches_the_gauss_newton_solution_with_more_iterations():
    """Both minimise J^h: the Picard (preconditioned gradient descent) solution agrees with
    the GN-PCG one to the solve tolerance, with far more outer iterations and PDE solves;
    the objective decreases monotonically."""
    P, _ = small_problem(shape=(16, 16), nt=8, reg=1, beta=1e-1)
    v_gn, rep_gn, S_gn = kr.gauss_newton(P, gtol=1e-4, max_outer=30)
    never = (10 ** 9, 0.0)   # no stagnation stop: only the gradient rule ends the iteration
    v_p, rep_p, S_p = kr.picard(P, gtol=1e-4, max_outer=2000, stagnation=never)
    assert rep_gn.converged and rep_p.converged and rep_p.reason == "relative gradient"
    assert np.abs(v_p - v_gn).max() <= 5e-3 * np.abs(v_gn).max()
    assert rep_p.iterations > 3 * rep_gn.iterations and rep_p.n_pde > rep_gn.n_pde
    assert all(b <= a for a, b in zip(rep_p.J, rep_p.J[1:]))
    _, rep_nm, _ = kr.picard(P, gtol=1e-4, max_outer=5000, memory=False, stagnation=never)
    assert rep_nm.iterations > rep_p.iterations       # the step-scale memory pays off
    _, rep_st, _ = kr.picard(P, gtol=1e-4, max_outer=2000)
    assert rep_st.reason == "objective stagnates" and rep_st.iterations < rep_p.iterations
