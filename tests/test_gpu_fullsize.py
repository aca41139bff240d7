"""Parity at the configurations' full sizes, in the launch configuration bench.py
times (captured matvec graphs), against the FP64 oracle where it finishes in
seconds and through properties that hold at any size where it does not (256^3).

FP32 tolerances: 1e-5 relative (L2) for m_1, the gradient at v = 0 and the
Hessian matvec; FP64: 1e-10 (rounding).
"""
import numpy as np
import pytest

import synth
from oracle import defgrad as odg
from oracle import krylov as okr
from oracle import reduced as ord_
from oracle import transport as otr
from tests.helpers import rel_inf, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_6299_amd as nk
    return nk


def dev_t(a, prec):
    dt = torch.float32 if prec == 32 else torch.float64
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda").to(dt).contiguous()


def dev_v(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def f32(a):
    """The values an FP32 transport sees (input images are rounded once on upload)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def kappa(P):
    """Cancellation factor of lambda = m_R - m_1: |m_T| / |m_R - m_T|."""
    return float(np.linalg.norm(P.mT) / np.linalg.norm(P.mR - P.mT))


def check_gradient_and_matvec_away_from_zero(G, P, v, w, prec):
    """Gradient and GN matvec at v != 0, where every v . grad term of the incremental
    and adjoint stages is active. FP64: 1e-10 elementwise. FP32: the GN matvec at 1e-5
    (relative L2); the gradient at 1e-5 max(1, kappa / 10) of the start-of-solve gradient
    scale, since lambda = m_R - m_1 amplifies the FP32 transport error by kappa."""
    S0 = ord_.objective_gradient(P, np.zeros(P.vshape()))
    S = ord_.objective_gradient(P, v)
    J, _, _, g = G.objective_gradient(dev_v(v))
    Hw = ord_.hessian_matvec(P, S, w)
    hw = host(G.hessian_matvec(dev_v(w)))
    gh = host(g)
    if prec == 64:
        assert abs(J - S.J) <= 1e-10 * abs(S.J)
        assert rel_inf(gh, S.g) < 1e-10
        assert rel_inf(hw, Hw) < 1e-10
    else:
        gscale = np.sqrt(np.sum(S0.g ** 2))
        assert np.sqrt(np.sum((gh - S.g) ** 2)) < 1e-5 * max(1.0, kappa(P) / 10.0) * gscale
        assert rel_l2(hw, Hw) < 1e-5


@pytest.fixture(scope="module")
def c2lit():
    spec = synth.CONFIGS["c2lit"]
    mT, vstar = synth.make_inputs(spec)
    mR = otr.forward_only(mT, vstar, spec.nt)
    P = ord_.Problem(mT, mR, spec.nt, 1, spec.reg, 0, spec.beta)
    S0 = ord_.objective_gradient(P, np.zeros(P.vshape()))
    w = synth.bandlimited_velocity(spec.shape, 20, 16, 0.02)
    Hw = ord_.hessian_matvec(P, S0, w)
    return spec, P, vstar, S0, w, Hw


@pytest.mark.parametrize("prec", [32, 64])
def test_c2lit_512_gradient_and_matvec(nk, c2lit, prec):
    """512^2, nt = 32, H2, beta = 1e-4: the bench workload."""
    spec, P, vstar, S0, w, Hw = c2lit
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=prec)
    G.set_images(dev_t(P.mT, prec), dev_t(P.mR, prec))
    tol = 1e-5 if prec == 32 else 1e-10
    m1 = host(G.forward(dev_v(vstar)))
    assert rel_l2(m1, P.mR) < tol
    J, Jd, Jr, g = G.objective_gradient(G.zeros_v())
    assert abs(J - S0.J) <= tol * abs(S0.J)
    assert rel_l2(host(g), S0.g) < tol
    out = G.empty_v()
    wt = dev_v(w)
    for _ in range(2):  # capture, then replay
        G.hessian_matvec(wt, out)
        assert rel_l2(host(out), Hw) < tol
    if prec == 64:
        assert rel_inf(host(g), S0.g) < tol and rel_inf(host(out), Hw) < tol
    G.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_c2lit_512_gradient_and_matvec_away_from_zero(nk, c2lit, prec):
    """512^2, nt = 32, H2: gradient and GN matvec at v = 0.5 v* (transport terms active)."""
    spec, P, vstar, S0, w, Hw = c2lit
    Pr = ord_.Problem(f32(P.mT), f32(P.mR), P.nt, 1, spec.reg, 0, spec.beta) if prec == 32 else P
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=prec)
    G.set_images(dev_t(P.mT, prec), dev_t(P.mR, prec))
    check_gradient_and_matvec_away_from_zero(G, Pr, 0.5 * vstar, w, prec)
    G.close()


def test_c2lit_512_autograd_fd_five_directions(nk, c2lit):
    """torch.autograd gradient (hand-written adjoint) vs central differences at 5 directions."""
    from paper_1408_6299_amd import objective
    spec, P, vstar, S0, w, Hw = c2lit
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=64)
    G.set_images(dev_t(P.mT, 64), dev_t(P.mR, 64))
    v0 = 0.5 * vstar
    vt = dev_v(v0).requires_grad_(True)
    objective(vt, G).backward()
    grad = vt.grad.detach()
    for seed in range(20, 25):
        d = synth.bandlimited_velocity(spec.shape, seed, 16, 0.01)
        eps = 1e-3
        fd = (G.objective(dev_v(v0 + eps * d))[0] - G.objective(dev_v(v0 - eps * d))[0]) / (2 * eps)
        an = float((grad * dev_v(d)).sum())
        assert abs(fd - an) <= 1e-6 * abs(an), (seed, fd, an)
    G.close()


def test_c2lit_512_fp32_solve_final_mismatch_matches_fp64(nk, c2lit):
    """The bench's time-to-solution run: beta continuation 1e-1 -> 1e-4 at 512^2, nt = 32,
    to a relative gradient of 1e-3 per level. The FP32 transport's final relative mismatch
    ||m_1 - m_R||^2 / ||m_T - m_R||^2 lies within 1e-4 (absolute) of the FP64 solve's. The
    FP64 library stands in for the oracle here (a CPU continuation at this size takes
    minutes); every FP64 operation of the path is pinned to the oracle to 1e-10 above."""
    spec, P, vstar, S0, w, Hw = c2lit
    mis = {}
    for prec in (64, 32):
        G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=prec)
        G.set_images(dev_t(P.mT, prec), dev_t(P.mR, prec))
        v, reps = G.continuation(spec.beta_levels, G.zeros_v(), gtol=1e-3, max_outer=50)
        assert all(r.converged for r in reps), prec
        m1 = host(G.forward(v))
        mis[prec] = float(np.sum((m1 - P.mR) ** 2) / np.sum((P.mT - P.mR) ** 2))
        G.close()
    assert mis[64] < 1e-2
    assert abs(mis[32] - mis[64]) <= 1e-4, mis


GOLDEN_C2 = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "c2lit_solve.json")


@pytest.mark.parametrize("prec", [32, 64])
def test_c2lit_512_solve_matches_the_oracle_solve(nk, c2lit, prec):
    """The bench's time-to-solution run against the FP64 oracle's continuation of the same
    512^2 workload (stored by tests/golden/make_c2lit_solve.py, which calls only the
    oracle): every level converges with the oracle's outer iterations to within one, and the
    final relative mismatch lies within 1e-4 (absolute) of the oracle's."""
    import json
    ref = json.load(open(GOLDEN_C2))
    spec, P, vstar, S0, w, Hw = c2lit
    assert list(spec.beta_levels) == ref["beta_levels"]
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=prec)
    G.set_images(dev_t(P.mT, prec), dev_t(P.mR, prec))
    v, reps = G.continuation(spec.beta_levels, G.zeros_v(), gtol=ref["gtol"], max_outer=50)
    for r, lv in zip(reps, ref["levels"]):
        assert r.converged and lv["converged"]
        assert abs(r.iterations - lv["iterations"]) <= 1, (r.iterations, lv)
    m1 = host(G.forward(v))
    mis = float(np.sum((m1 - P.mR) ** 2) / np.sum((P.mT - P.mR) ** 2))
    assert abs(mis - ref["relative_mismatch"]) <= 1e-4, (mis, ref["relative_mismatch"])
    G.close()


GOLDEN_BS = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "c2beta_search.json")


@pytest.mark.parametrize("prec", [64, 32])
def test_c2beta_256_beta_search_matches_the_oracle_search(nk, prec):
    """The bench's beta search (256^2, nt = 64, H1, bound eps_F on det F_1) against the FP64
    oracle's search of the same workload (stored by tests/golden/make_c2beta_search.py, which
    calls only the oracle). FP64: the same trials and decisions, min det F_1 per trial within
    1e-8 and the same beta*. FP32: every decision follows the bound and beta* lies within two
    bisection steps of the oracle's."""
    import json
    ref = json.load(open(GOLDEN_BS))
    spec = synth.CONFIGS["c2beta"]
    mT, vstar = synth.make_inputs(spec)
    mR = otr.forward_only(mT, vstar, spec.nt)   # the reference image, as the stored search used
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, 1.0, precision=prec)
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    v, res = G.beta_search(ref["eps_F"], gtol=ref["gtol"], max_outer=50)
    assert res.breached == ref["breached"] and res.reason == ref["reason"]
    for t in res.trials:
        assert (t.min_det >= ref["eps_F"]) == t.accepted
    if prec == 64:
        assert [t.beta for t in res.trials] == [r["beta"] for r in ref["trials"]]
        assert [t.accepted for t in res.trials] == [r["accepted"] for r in ref["trials"]]
        for t, r in zip(res.trials, ref["trials"]):
            assert abs(t.min_det - r["min_det"]) < 1e-8, (t, r)
        assert res.beta_star == ref["beta_star"]
    else:
        assert abs(res.beta_star - ref["beta_star"]) <= 2 * ref["dbeta_min"]
    G.close()


GOLDEN_SOLVERS = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "c2lit_solvers.json")


@pytest.mark.parametrize("prec", [64, 32])
def test_c2lit_512_gn_and_picard_match_the_oracle(nk, c2lit, prec):
    """GN-PCG and the globalised Picard iteration (with and without the stagnation stop) at
    beta = 1e-2 on the headline grid, from v = 0 to a relative gradient of 1e-3, against the
    FP64 oracle's runs (stored by tests/golden/make_c2lit_solvers.py, oracle calls only).
    The stop reason and the final objective agree; the iteration and PDE-solve counts agree
    exactly in FP64 for GN-PCG and to within a few percent otherwise, since the inexact inner
    solves and Picard's line search and step memory turn rounding into occasional one-step
    differences."""
    import json
    ref = json.load(open(GOLDEN_SOLVERS))
    spec, P, vstar, S0, w, Hw = c2lit
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, ref["beta"], precision=prec)
    G.set_images(dev_t(P.mT, prec), dev_t(P.mR, prec))
    runs = {"gn_pcg": lambda: G.newton_solve(G.zeros_v(), gtol=ref["gtol"], max_outer=50),
            "picard": lambda: G.picard_solve(G.zeros_v(), gtol=ref["gtol"], max_outer=2000),
            "picard_no_stagnation_stop": lambda: G.picard_solve(G.zeros_v(), gtol=ref["gtol"], max_outer=2000,
                                                                stagnation=(0, 0.0))}
    for name, run in runs.items():
        r = ref[name]
        _, rep = run()
        assert rep.converged == r["converged"], name
        got = {"outer": rep.iterations, "n_pde": rep.n_pde}
        want = {"outer": r["outer_iterations"], "n_pde": r["n_pde"]}
        if prec == 64 and name == "gn_pcg":
            assert got == want, (name, got, want)
        else:
            for k in got:
                assert abs(got[k] - want[k]) <= max(1, 0.05 * want[k]), (name, got, want)
        assert abs(rep.J - r["J"]) <= 1e-4 * abs(r["J"]), (name, rep.J, r["J"])
    G.close()


GOLDEN_NEWTON = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                           "c2lit_newton_solve.json")


@pytest.mark.parametrize("prec", [64, 32])
def test_c2lit_512_full_newton_solve_matches_the_oracle_solve(nk, c2lit, prec):
    """The bench's full-Newton continuation (512^2, nt = 32) against the FP64 oracle's
    (stored by tests/golden/make_c2lit_newton_solve.py, oracle calls only): every level
    converges with the oracle's outer iterations to within one, and the final relative
    mismatch lies within 1e-4 (absolute) of the oracle's."""
    import json
    ref = json.load(open(GOLDEN_NEWTON))
    spec, P, vstar, S0, w, Hw = c2lit
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=prec)
    G.hessian = "newton"
    G.set_images(dev_t(P.mT, prec), dev_t(P.mR, prec))
    v, reps = G.continuation(spec.beta_levels, G.zeros_v(), gtol=ref["gtol"], max_outer=50)
    for r, lv in zip(reps, ref["levels"]):
        assert r.converged and lv["converged"]
        assert abs(r.iterations - lv["iterations"]) <= 1, (r.iterations, lv)
    m1 = host(G.forward(v))
    mis = float(np.sum((m1 - P.mR) ** 2) / np.sum((P.mT - P.mR) ** 2))
    assert abs(mis - ref["relative_mismatch"]) <= 1e-4, (mis, ref["relative_mismatch"])
    G.close()


def test_c0_64_gauss_newton_solve_matches_oracle(nk):
    """64^2 FP64, H1, beta = 1e-2, nt = 16: the whole GN-PCG solve to relative gradient 1e-3."""
    spec = synth.CONFIGS["c0"]
    mT, vstar = synth.make_inputs(spec)
    mR = otr.forward_only(mT, vstar, spec.nt)
    P = ord_.Problem(mT, mR, spec.nt, 1, spec.reg, 0, spec.beta)
    v_ref, rep_ref, S_ref = okr.gauss_newton(P, gtol=1e-3, max_outer=50)
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=64)
    G.set_images(dev_t(mT, 64), dev_t(mR, 64))
    v, rep = G.newton_solve(gtol=1e-3, max_outer=50)
    assert rep.converged and rep_ref.converged
    assert rep.iterations == rep_ref.iterations
    assert rep.cg_iterations == rep_ref.matvecs
    assert rel_inf(host(v), v_ref) < 1e-8
    mis0 = np.sum((mR - mT) ** 2)
    assert abs(2 * rep.J_dist / (P.hd * mis0) - 2 * S_ref.J_dist / (P.hd * mis0)) < 1e-4
    G.close()


def test_c1_256_three_coefficients_stokes(nk):
    """256^2, n_c = 3 Chebyshev coefficients, H2 + Stokes, beta = 1e-3, nt = 408, FP32 and FP64."""
    spec = synth.CONFIGS["c1"]
    mT, vstar = synth.make_inputs(spec)
    mR = otr.forward_only(mT, vstar, spec.nt)
    P = ord_.Problem(mT, mR, spec.nt, spec.nc, spec.reg, 1, spec.beta)
    S0 = ord_.objective_gradient(P, np.zeros(P.vshape()))
    w = synth.bandlimited_velocity(spec.shape, 30, 8, 0.1, divfree=True, nc=3)
    Hw = ord_.hessian_matvec(P, S0, w)
    for prec in (32, 64):
        tol = 1e-5 if prec == 32 else 1e-10
        G = nk.Problem(spec.shape, spec.nt, spec.nc, spec.reg, True, spec.beta, precision=prec)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        J, _, _, g = G.objective_gradient(G.zeros_v())
        assert rel_l2(host(g), S0.g) < tol
        assert rel_l2(host(G.hessian_matvec(dev_v(w))), Hw) < tol
        G.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_c1_256_three_coefficients_stokes_away_from_zero(nk, prec):
    """256^2, n_c = 3, H2 + Stokes, nt = 408: gradient and GN matvec at v = 0.5 v*."""
    spec = synth.CONFIGS["c1"]
    mT, vstar = synth.make_inputs(spec)
    mR = otr.forward_only(mT, vstar, spec.nt)
    if prec == 32:
        mT, mR = f32(mT), f32(mR)
    P = ord_.Problem(mT, mR, spec.nt, spec.nc, spec.reg, 1, spec.beta)
    w = synth.bandlimited_velocity(spec.shape, 30, 8, 0.1, divfree=True, nc=3)
    G = nk.Problem(spec.shape, spec.nt, spec.nc, spec.reg, True, spec.beta, precision=prec)
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    check_gradient_and_matvec_away_from_zero(G, P, 0.5 * vstar, w, prec)
    G.close()


def test_c1_256_det_grad_y_of_divergence_free_velocity(nk):
    """det F_1 statistics in FP64 for the three-coefficient divergence-free velocity."""
    spec = synth.CONFIGS["c1"]
    _, vstar = synth.make_inputs(spec)
    nt = 64  # the oracle's cost grows with nt; the statistic is a parity check, not a convergence study
    ref_det, ref_stats = odg.det_stats(vstar, nt)
    G = nk.Problem(spec.shape, nt, spec.nc, spec.reg, True, spec.beta, precision=32)
    det, stats = G.det_grad_y(dev_v(vstar))
    assert np.abs(host(det) - ref_det).max() < 1e-10
    assert np.allclose(stats, ref_stats, rtol=0, atol=1e-10)
    assert abs(stats[0] - 1) < 1e-2 and abs(stats[1] - 1) < 1e-2
    G.close()


def test_c3_batch_subset(nk):
    """Batched workload: every grid size of the 64-item batch, one graph launch, equal to
    single-item matvecs bit for bit; one item of every grid size (64^2 to 512^2) against the
    oracle."""
    specs = synth.batch_specs()
    picks, seen = [], set()
    for i, sp in enumerate(specs):
        if sp.shape[0] not in seen:
            seen.add(sp.shape[0])
            picks.append(i)
    picks += [i for i in range(len(specs)) if i not in picks][:4]
    probs, ws, refs, host_items = [], [], [], []
    for i in picks:
        sp = specs[i]
        mT, vstar = synth.make_inputs(sp)
        G = nk.Problem(sp.shape, sp.nt, 1, sp.reg, False, sp.beta, precision=32)
        mR = otr.forward_only(mT, vstar, sp.nt)   # the reference image: the oracle's forward solve
        G.set_images(dev_t(mT, 32), dev_t(mR, 32))
        G.objective_gradient(G.zeros_v())
        w = synth.bandlimited_velocity(sp.shape, 500 + i, 6, 0.05)
        probs.append(G)
        ws.append(dev_v(w))
        refs.append(host(G.hessian_matvec(ws[-1])))
        host_items.append((mT, mR, w, sp))
    B = nk.Batch(probs)
    for _ in range(2):
        outs = B.hessian_matvec(ws)
        for o, r in zip(outs, refs):
            assert np.array_equal(host(o), r)
    # The kernels transport the FP32-rounded images, so the oracle takes those (its
    # arithmetic stays FP64); the GN matvec does not involve lambda, so the plain FP32
    # bound holds at every grid size.
    for k in range(len(seen)):                  # the first pick of each grid size
        mT, mR, w, sp = host_items[k]
        P = ord_.Problem(f32(mT), f32(mR), sp.nt, 1, sp.reg, 0, sp.beta)
        S0 = ord_.objective_gradient(P, np.zeros(P.vshape()))
        assert rel_l2(refs[k], ord_.hessian_matvec(P, S0, w)) < 1e-5, sp.shape


def test_c3_cfl_step_items_share_launches_and_match_the_oracle(nk):
    """Items of the CFL-step batch (each with the steps its own CFL bound needs): 64^2 and
    128^2 items of two step counts each join one group per grid size, equal their own
    matvecs bit for bit at v = 0.5 v*, and one item of every (grid, nt) pair matches the
    oracle there (FP32-rounded inputs, the FP32 bound)."""
    specs = synth.batch_specs_nteff()
    picks = {}
    for i, sp in enumerate(specs):
        key = (sp.shape[0], sp.nt)
        if sp.shape[0] in (64, 128) and key not in picks and sum(k[0] == sp.shape[0] for k in picks) < 2:
            picks[key] = i
    assert sorted({k[0] for k in picks}) == [64, 128] and len(picks) == 4, picks
    probs, ws, vs, refs, data = [], [], [], [], []
    for (n, nt), i in sorted(picks.items()):
        sp = specs[i]
        mT, vstar = synth.make_inputs(sp)
        mR = otr.forward_only(mT, vstar, sp.nt)
        G = nk.Problem(sp.shape, sp.nt, 1, sp.reg, False, sp.beta, precision=32)
        G.set_images(dev_t(mT, 32), dev_t(mR, 32))
        v = 0.5 * vstar
        G.objective_gradient(dev_v(v))
        w = synth.bandlimited_velocity(sp.shape, 500 + i, 6, 0.05)
        probs.append(G)
        ws.append(dev_v(w))
        refs.append(host(G.hessian_matvec(ws[-1])))
        data.append((mT, mR, v, w, sp))
    B = nk.Batch(probs)
    for _ in range(2):
        outs = B.hessian_matvec(ws)
        for o, r in zip(outs, refs):
            assert np.array_equal(host(o), r)
    assert sorted(n for n, _ in B.group_plan()) == [2, 2], B.group_plan()
    B.close()
    for (mT, mR, v, w, sp), ref, G in zip(data, refs, probs):
        P = ord_.Problem(f32(mT), f32(mR), sp.nt, 1, sp.reg, 0, sp.beta)
        S = ord_.objective_gradient(P, v)
        assert rel_l2(ref, ord_.hessian_matvec(P, S, f32(w).astype(np.float64))) < 1e-5, (sp.shape, sp.nt)
        G.close()


def test_c3_512_batch_item_away_from_zero(nk):
    """The first 512^2 item of the 64-pair batch (FP32, H1, nt = 16): gradient and GN
    matvec at v = 0.5 v* against the oracle, alone and through a batch of itself and a
    second item (bit-identical)."""
    specs = synth.batch_specs()
    i = next(k for k, sp in enumerate(specs) if sp.shape[0] == 512)
    sp = specs[i]
    mT, vstar = synth.make_inputs(sp)
    mR = otr.forward_only(mT, vstar, sp.nt)
    P = ord_.Problem(f32(mT), f32(mR), sp.nt, 1, sp.reg, 0, sp.beta)
    w = synth.bandlimited_velocity(sp.shape, 500 + i, 6, 0.05)
    G = nk.Problem(sp.shape, sp.nt, 1, sp.reg, False, sp.beta, precision=32)
    G.set_images(dev_t(mT, 32), dev_t(mR, 32))
    check_gradient_and_matvec_away_from_zero(G, P, 0.5 * vstar, w, 32)
    single = host(G.hessian_matvec(dev_v(w)))
    H = nk.Problem(sp.shape, sp.nt, 1, sp.reg, False, sp.beta, precision=32)
    H.set_images(dev_t(mT, 32), dev_t(mR, 32))
    H.objective_gradient(dev_v(0.5 * vstar))
    B = nk.Batch([G, H])
    outs = B.hessian_matvec([dev_v(w), dev_v(w)])
    assert np.array_equal(host(outs[0]), single) and np.array_equal(host(outs[1]), single)
    G.close()
    H.close()


def test_c4_64cube_oracle_parity(nk):
    """The 3D generator (smooth image, divergence-free band-limited velocity, H2 + Stokes)
    at 64^3, nt = 32, checkpointing every 8 steps, against the oracle."""
    spec = synth.CONFIGS["c4"]
    shape = (64, 64, 64)
    mT = synth.smooth_image(shape, spec.image_seed, spec.image_width / 16.0)
    vstar = synth.bandlimited_velocity(shape, spec.vel_seed, 4, synth.cfl_literal_linf(64, 32), divfree=True,
                                       norm="linf")
    mR = otr.forward_only(mT, vstar, spec.nt)
    P = ord_.Problem(mT, mR, spec.nt, 1, spec.reg, 1, spec.beta)
    S0 = ord_.objective_gradient(P, np.zeros(P.vshape()))
    w = synth.bandlimited_velocity(shape, 41, 4, 0.05, divfree=True)
    Hw = ord_.hessian_matvec(P, S0, w)
    for prec in (32, 64):
        tol = 1e-5 if prec == 32 else 1e-10
        G = nk.Problem(shape, spec.nt, 1, spec.reg, True, spec.beta, precision=prec, checkpoint_every=8)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        _, _, _, g = G.objective_gradient(G.zeros_v())
        assert rel_l2(host(g), S0.g) < tol
        assert rel_l2(host(G.hessian_matvec(dev_v(w))), Hw) < tol
        G.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_c4_256cube_full_grid_against_the_oracle(nk, prec):
    """The 256^3 grid itself against the oracle, over a short horizon the oracle finishes
    in about a minute: H2 + Stokes, beta 1e-3, nt = 2 with the C4 generators (velocity at
    CFL 0.1 for two steps), FP32 with the trajectory checkpointed every step (two segments,
    one slot, so every sweep recomputes one). Gradient and GN matvec at v = 0.5 v*, and the
    first PCG solve of the Newton step at two fixed iterations. FP64: 1e-10 (PCG 1e-9);
    FP32: the GN matvec at 1e-5, the gradient at the kappa-scaled bound, PCG at 1e-4."""
    spec = synth.CONFIGS["c4"]
    shape, nt = spec.shape, 2
    mT = synth.smooth_image(shape, spec.image_seed, spec.image_width)
    vstar = synth.bandlimited_velocity(shape, spec.vel_seed, spec.vel_kmax, synth.cfl_literal_linf(256, nt),
                                       divfree=True, norm="linf")
    mR = otr.forward_only(mT, vstar, nt)
    if prec == 32:
        mT, mR = f32(mT), f32(mR)
    P = ord_.Problem(mT, mR, nt, 1, spec.reg, 1, spec.beta)
    v = 0.5 * vstar
    w = synth.bandlimited_velocity(shape, 41, 6, 0.05, divfree=True)
    G = nk.Problem(shape, nt, 1, spec.reg, True, spec.beta, precision=prec, checkpoint_every=1 if prec == 32 else 0)
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    check_gradient_and_matvec_away_from_zero(G, P, v, w, prec)
    S = ord_.objective_gradient(P, v)
    x_ref, it_ref, _, _ = okr.pcg(lambda q: ord_.hessian_matvec(P, S, q), lambda r: ord_.precond(P, r), -S.g, 0.0, 2)
    _, _, _, g = G.objective_gradient(dev_v(v))
    x, it, _, _ = G.pcg((-g).contiguous(), 0.0, 2)
    assert it == it_ref == 2
    assert rel_inf(host(x), x_ref) < (1e-9 if prec == 64 else 1e-4)
    G.close()


def test_c4_256cube_properties(nk):
    """256^3 FP32, H2 + Stokes, beta = 1e-3, nt = 32, checkpoint every 8: the oracle cannot run
    here, so check what holds at any size: a constant image stays constant, checkpointing is
    exact, the GN Hessian is symmetric, FP32 agrees with FP64, and det F_1 = 1 for the
    divergence-free velocity to O(h_t^2)."""
    spec = synth.CONFIGS["c4"]
    shape, nt = spec.shape, spec.nt
    mT, vstar = synth.make_inputs(spec)
    G32 = nk.Problem(shape, nt, 1, spec.reg, True, spec.beta, precision=32, checkpoint_every=8)
    const = torch.full(shape, 0.37, dtype=torch.float32, device="cuda")
    G32.set_images(const, const)
    m1 = G32.forward(dev_v(vstar))
    assert float((m1 - 0.37).abs().max()) < 1e-6
    # reference image from the library's FP64 forward solve (input synthesis, not a check)
    G64 = nk.Problem(shape, nt, 1, spec.reg, True, spec.beta, precision=64, checkpoint_every=8)
    G64.set_images(dev_t(mT, 64), torch.zeros(shape, dtype=torch.float64, device="cuda"))
    mR = G64.forward(dev_v(vstar))
    G64.set_images(dev_t(mT, 64), mR)
    G32.set_images(dev_t(mT, 32), mR.float())
    _, _, _, g64 = G64.objective_gradient(G64.zeros_v())
    _, _, _, g32 = G32.objective_gradient(G32.zeros_v())
    assert rel_l2(host(g32), host(g64)) < 1e-5
    u = dev_v(synth.bandlimited_velocity(shape, 51, 6, 0.05, divfree=True))
    w = dev_v(synth.bandlimited_velocity(shape, 52, 6, 0.05, divfree=True))
    Hu64, Hw64 = G64.hessian_matvec(u), G64.hessian_matvec(w)
    a, b = float((u * Hw64).sum()), float((Hu64 * w).sum())
    assert abs(a - b) <= 1e-12 * abs(a)
    Hw32 = G32.hessian_matvec(w)
    assert rel_l2(host(Hw32), host(Hw64)) < 1e-5
    det, stats = G32.det_grad_y(dev_v(vstar))
    assert abs(stats[0] - 1) < 1e-3 and abs(stats[1] - 1) < 1e-3 and abs(stats[2] - 1) < 1e-4
    G32.close()
    G64.close()


def test_largest_grid_512cube_closed_form_and_symmetry(nk):
    """The largest grid the library takes (512^3, FP32, nt = 2). A constant velocity moves
    each Fourier mode by the Heun factor G(z) = 1 + z + z^2/2 per step, z = -i h (k . v),
    so m_T = sin(x1) + cos(3 x3) under v = (a1, 0, a3) ends as
    Im(G(-i h a1)^nt e^{i x1}) + Re(G(-3 i h a3)^nt e^{3 i x3}) at every point (the
    constant-velocity closed form the oracle is pinned to). The GN Hessian at that state is
    symmetric for two smooth directions to FP32 rounding."""
    n, nt = 512, 2
    shape = (n, n, n)
    h = 1.0 / nt
    a1, a3 = 0.004, -0.003
    x = torch.arange(n, dtype=torch.float64, device="cuda") * (2 * np.pi / n)
    X1 = x.view(n, 1, 1)
    X3 = x.view(1, 1, n)
    mT = (torch.sin(X1) + torch.cos(3 * X3)).expand(shape).contiguous()
    G = nk.Problem(shape, nt, 1, 1, False, 1e-2, precision=32)
    v = torch.zeros(G.vshape, dtype=torch.float64, device="cuda")
    v[0, 0] = a1
    v[0, 2] = a3
    G.set_images(mT.float(), mT.float())
    m1 = G.forward(v)
    heun = lambda z: (1 + z + z * z / 2) ** nt
    g1, g3 = heun(-1j * h * a1), heun(-3j * h * a3)
    ref = (abs(g1) * torch.sin(X1 + np.angle(g1)) + abs(g3) * torch.cos(3 * X3 + np.angle(g3))).expand(shape)
    err = float((m1.double() - ref).abs().max())
    moved = float((ref - mT).abs().max())   # how far the closed form is from the template
    assert err < 5e-6 and moved > 1e-3, (err, moved)
    del ref, m1
    # reference image: the template moved by the velocity (library forward, input synthesis)
    mR = G.forward(2.0 * v)
    G.set_images(mT.float(), mR)
    G.objective_gradient(v)
    X2 = x.view(1, n, 1)
    u = torch.zeros_like(v)
    u[0, 0] = 0.01 * torch.sin(X2)
    u[0, 1] = 0.01 * torch.cos(X3)
    u[0, 2] = 0.01 * torch.sin(X1)
    w = u.clone()                       # w = u + r keeps <u, Hw> away from zero (H is SPD)
    w[0, 0] += 0.005 * torch.cos(2 * X3)
    w[0, 1] += 0.005 * torch.sin(X1)
    w[0, 2] += 0.005 * torch.cos(X2)
    Hw = G.hessian_matvec(w)
    Hu = G.hessian_matvec(u)
    s1, s2 = float((u * Hw).sum()), float((Hu * w).sum())
    assert abs(s1 - s2) <= 1e-5 * abs(s1), (s1, s2)
    assert torch.isfinite(Hw).all()
    G.close()
