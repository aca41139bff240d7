"""GPU (HIP, gfx950) vs FP64 oracle parity, element by element, through the C ABI.

Tolerances: FP64 GPU vs oracle to rounding (<= 1e-10 relative, max norm); FP32
transport vs the FP64 oracle to <= 1e-5 relative (L2), with the gradient's
bound scaled by the mismatch cancellation factor as explained in the test.
"""
import numpy as np
import pytest

import synth
from oracle import defgrad as odg
from oracle import krylov as okr
from oracle import reduced as ord_
from oracle import spectral as osp
from oracle import transport as otr
from tests.helpers import rel_inf, rel_l2, smooth_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {64: 1e-10, 32: 1e-5}


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_6299_amd as nk
    return nk


def dev_t(a, prec):
    """A scalar field in the transport precision."""
    dt = torch.float32 if prec == 32 else torch.float64
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda").to(dt).contiguous()


def dev_v(a):
    """A velocity-shaped array (always FP64)."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def test_single_hip_runtime_in_process(nk):
    """The library binds to torch's HIP runtime: one libamdhip64 mapped, and it works."""
    maps = open("/proc/self/maps").read().splitlines()
    hip = {l.split()[-1] for l in maps if "libamdhip64" in l}
    nkreg = {l.split()[-1] for l in maps if "libnkreg" in l}
    assert len(hip) == 1, hip
    assert len(nkreg) == 1 and next(iter(nkreg)).startswith(
        __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__))))
    p = nk.Problem((8, 8), 2, precision=64)
    p.close()


SHAPES = [(8, 8), (16, 32), (64, 64), (8, 16, 8), (16, 8, 32)]


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("shape", SHAPES)
def test_gradient_and_divergence(nk, shape, prec):
    rng = np.random.default_rng(1)
    u = rng.standard_normal(shape)
    w = rng.standard_normal((len(shape),) + shape)
    p = nk.Problem(shape, 4, precision=prec)
    g = host(p.gradient(dev_t(u, prec)))
    assert rel_inf(g, osp.grad(u)) < (1e-12 if prec == 64 else 2e-6)
    s = host(p.divergence(dev_t(w, prec)))
    assert rel_inf(s, osp.div(w)) < (1e-12 if prec == 64 else 2e-6)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("shape,nc,reg", [((8, 8), 1, 1), ((32, 16), 2, 2), ((8, 16, 8), 1, 2), ((16, 16, 8), 2, 1)])
def test_spectral_operators(nk, shape, nc, reg, prec):
    rng = np.random.default_rng(2)
    d = len(shape)
    x = rng.standard_normal((nc, d) + shape)
    beta = 3e-3
    p = nk.Problem(shape, 4, nc=nc, reg=reg, beta=beta, precision=prec)
    tol = 1e-12 if prec == 64 else 3e-6
    assert rel_inf(host(p.apply_reg(dev_v(x))), osp.apply_A(x, reg, d)) < tol
    assert rel_inf(host(p.precond(dev_v(x))), osp.apply_Pinv(x, reg, beta, d)) < tol
    ref_k = np.stack([osp.apply_K(x[l]) for l in range(nc)])
    assert rel_inf(host(p.project(dev_v(x))), ref_k) < tol


def make_pair(nk, shape, nt, nc, reg, gamma, beta, prec, vscale=0.5):
    mT, mR, vstar, w = smooth_inputs(shape, nt, nc=nc, divfree=bool(gamma))
    P = ord_.Problem(mT, mR, nt, nc, reg, gamma, beta)
    G = nk.Problem(shape, nt, nc=nc, reg=reg, incompressible=bool(gamma), beta=beta, precision=prec)
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    return P, G, vscale * vstar, w


CASES = [
    # shape, nt, nc, reg, gamma, beta
    ((16, 16), 6, 1, 1, 0, 1e-2),
    ((64, 64), 16, 1, 1, 0, 1e-2),
    ((32, 64), 8, 3, 2, 1, 1e-3),
    ((8, 16, 8), 4, 1, 2, 1, 1e-3),
    ((16, 8, 16), 6, 2, 1, 0, 1e-2),
]


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("case", CASES)
def test_forward_objective_gradient_matvec(nk, case, prec):
    shape, nt, nc, reg, gamma, beta = case
    P, G, v, w = make_pair(nk, shape, nt, nc, reg, gamma, beta, prec)
    tol = TOL[prec]
    # state equation
    m1 = host(G.forward(dev_v(v)))
    ref_m1 = otr.forward_only(P.mT, v, nt)
    assert rel_inf(m1, ref_m1) < tol
    # objective and reduced gradient; first at v = 0 (start of the solve), then at v.
    # In FP32 the error of g is the FP32 error of the transported image amplified by
    # the cancellation in lambda = m_R - m_1, by kappa = |m_T| / |m_R - m_T|; it is
    # measured against the gradient scale at the start of the solve (the scale of the
    # relative-gradient stopping rule) with tolerance 1e-5 * max(1, kappa / 10).
    S0 = ord_.objective_gradient(P, np.zeros_like(v))
    _, _, _, g0 = G.objective_gradient(dev_v(np.zeros_like(v)))
    assert rel_l2(host(g0), S0.g) < tol
    S = ord_.objective_gradient(P, v)
    J, Jd, Jr, g = G.objective_gradient(dev_v(v))
    assert abs(J - S.J) <= (1e-10 if prec == 64 else 1e-4) * abs(S.J)
    assert abs(Jr - S.J_reg) <= (1e-10 if prec == 64 else 1e-5) * abs(S.J_reg)
    gscale = np.sqrt(np.sum(S0.g ** 2))
    kappa = np.linalg.norm(P.mT) / np.linalg.norm(P.mR - P.mT)
    gtol = tol if prec == 64 else tol * max(1.0, kappa / 10.0)
    assert np.sqrt(np.sum((host(g) - S.g) ** 2)) < gtol * gscale
    if prec == 64:
        assert rel_inf(host(g), S.g) < tol
    # Gauss-Newton Hessian matvec
    hw = host(G.hessian_matvec(dev_v(w)))
    ref = ord_.hessian_matvec(P, S, w)
    assert rel_inf(hw, ref) < (tol if prec == 64 else 2e-5)
    assert rel_l2(hw, ref) < tol
    G.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_pcg_fixed_iterations_matches_oracle(nk, prec):
    shape, nt, nc, reg, gamma, beta = (32, 32), 8, 1, 2, 0, 1e-2
    P, G, v, w = make_pair(nk, shape, nt, nc, reg, gamma, beta, prec)
    S = ord_.objective_gradient(P, v)
    _, _, _, g = G.objective_gradient(dev_v(v))
    rhs = -S.g
    for maxit in (1, 4):
        x_ref, it_ref, rr_ref, _ = okr.pcg(lambda q: ord_.hessian_matvec(P, S, q),
                                           lambda r: ord_.precond(P, r), rhs, 0.0, maxit)
        s, it, rr, conv = G.pcg(dev_v(rhs), 0.0, maxit)
        assert it == it_ref == maxit and not conv
        assert rel_inf(host(s), x_ref) < (1e-9 if prec == 64 else 1e-4)
        assert abs(rr - rr_ref) <= (1e-8 if prec == 64 else 1e-4) * rr_ref
    s, it, rr, conv = G.pcg(dev_v(rhs), 1e-2, 0)
    assert conv and rr <= 1e-2


@pytest.mark.parametrize("shape,nc,divfree", [((32, 32), 1, False), ((32, 32), 3, True), ((8, 16, 8), 1, True)])
def test_det_grad_y(nk, shape, nc, divfree):
    """det F_1 runs in FP64 in both modes (velocities are FP64 arrays)."""
    nt = 8
    v = synth.bandlimited_velocity(shape, 12, 3, 0.8, divfree=divfree, nc=nc)
    ref_det, ref_stats = odg.det_stats(v, nt)
    for prec in (64, 32):
        G = nk.Problem(shape, nt, nc=nc, precision=prec)
        det, stats = G.det_grad_y(dev_v(v))
        assert np.abs(host(det) - ref_det).max() < 1e-10
        assert np.allclose(stats, ref_stats, rtol=0, atol=1e-10)


def test_call_order_and_cfl_errors(nk):
    shape, nt = (16, 16), 4
    G = nk.Problem(shape, nt, precision=64, cfl_max=0.2)
    mT, mR, vstar, w = smooth_inputs(shape, nt)
    with pytest.raises(nk.NkregError) as ei:
        G.forward(dev_v(vstar))
    assert ei.value.status == -5  # no images yet
    G.set_images(dev_t(mT, 64), dev_t(mR, 64))
    with pytest.raises(nk.NkregError) as ei:
        G.hessian_matvec(dev_v(w))
    assert ei.value.status == -5
    big = np.zeros((1, 2) + shape)
    big[0, 0] = 10.0  # CFL number 10 * 16 / (2 pi) / 4 >> 0.2
    with pytest.raises(nk.NkregError) as ei:
        G.objective_gradient(dev_v(big))
    assert ei.value.status == -7
    nanimg = mT.copy()
    nanimg[3, 3] = np.nan
    # a non-finite template is refused on upload (its mean centres both images) ...
    with pytest.raises(nk.NkregError) as ei:
        G.set_images(dev_t(nanimg, 64), dev_t(mR, 64))
    assert ei.value.status == -6
    # ... a non-finite reference image when the objective is evaluated
    G.set_images(dev_t(mT, 64), dev_t(nanimg, 64))
    with pytest.raises(nk.NkregError) as ei:
        G.objective_gradient(dev_v(0 * vstar))
    assert ei.value.status == -6


# (shape, nt, precision, beta, seed, checkpoint): items 0-2 share a group (beta and data
# differ per item), 3-4 another, 5 differs only in nt (it joins items 0-2 with inactive
# entries for the steps it does not take), 6-7 are 3D Stokes with checkpointing, 8 is FP64.
BATCH_ITEMS = [((32, 32), 6, 32, 1e-2, 1, 0), ((32, 32), 6, 32, 1e-3, 2, 0), ((32, 32), 6, 32, 3e-2, 3, 0),
               ((64, 32), 8, 32, 1e-2, 4, 0), ((64, 32), 8, 32, 1e-2, 5, 0), ((32, 32), 4, 32, 1e-2, 6, 0),
               ((16, 8, 16), 6, 32, 1e-3, 7, 4), ((16, 8, 16), 6, 32, 1e-3, 8, 4), ((32, 32), 6, 64, 1e-2, 9, 0)]


def test_batch_matches_single_items(nk):
    """Items of one configuration share each kernel launch (per-item pointers and beta from
    a device table); the batched result equals every item's own matvec bit for bit, on
    the first build and on replays, also after one item's beta changes."""
    probs, ws, refs = [], [], []
    for shape, nt, prec, beta, seed, ck in BATCH_ITEMS:
        gamma = len(shape) == 3
        mT, mR, vstar, w = smooth_inputs(shape, nt, divfree=gamma, seed=seed)
        G = nk.Problem(shape, nt, reg=2 if gamma else 1, incompressible=gamma, beta=beta, precision=prec,
                       checkpoint_every=ck)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        G.objective_gradient(dev_v(0.5 * vstar))
        probs.append(G)
        ws.append(dev_v(w))
        refs.append(host(G.hessian_matvec(ws[-1])))
    B = nk.Batch(probs)
    outs = [p.empty_v() for p in probs]
    for _ in range(3):
        B.hessian_matvec(ws, outs)
        for o, r in zip(outs, refs):
            assert np.array_equal(host(o), r)
    # four groups; the 64 x 32 pair may take the tiled column pass (timed at group scale),
    # the others have no axis it applies to
    plan = B.group_plan()
    assert sorted(n for n, _ in plan) == [1, 2, 2, 4]
    assert sum(f == "tiled" for _, f in plan) <= 1
    assert all(f in nk.Batch.GROUP_FORMS for _, f in plan)
    # a beta change invalidates the graph; the rebuilt batch uses the new beta for that item
    probs[1].beta = 5e-3
    ref1 = host(probs[1].hessian_matvec(ws[1]))
    assert not np.array_equal(ref1, refs[1])
    B.hessian_matvec(ws, outs)
    assert np.array_equal(host(outs[1]), ref1)
    for i in (0, 2, 3, 8):
        assert np.array_equal(host(outs[i]), refs[i])
    B.close()
    for p in probs:
        p.close()


def test_batch_created_from_configs_gradient_and_state_match_single_items(nk):
    """nkreg_batch_create from configurations (the batch owns its items), each item's
    images set through its handle; one batched objective-and-gradient call equals every
    item's own nkreg_objective_gradient bit for bit (J and g), on the first build and on a
    replay at new velocities; nkreg_batch_set_state leaves the states the batched matvec
    then uses, equal to single items' matvecs bit for bit. One FP64 item of each grid
    against the oracle at 1e-10."""
    cfgs, data = [], []
    for shape, nt, prec, beta, seed, ck in BATCH_ITEMS:
        gamma = len(shape) == 3
        mT, mR, vstar, w = smooth_inputs(shape, nt, divfree=gamma, seed=seed)
        cfgs.append(dict(shape=shape, nt=nt, reg=2 if gamma else 1, incompressible=gamma, beta=beta,
                         precision=prec, checkpoint_every=ck))
        data.append((mT, mR, vstar, w, prec))
    B = nk.Batch.create(cfgs)
    singles = []
    for item, c, (mT, mR, vstar, w, prec) in zip(B.items, cfgs, data):
        item.set_images(dev_t(mT, prec), dev_t(mR, prec))
        G = nk.Problem(**c)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        singles.append(G)
    for scale in (0.5, 0.25):
        vs = [dev_v(scale * d[2]) for d in data]
        J, Jd, Jr, gs = B.objective_gradient(vs)
        for i, G in enumerate(singles):
            Ji, Jdi, Jri, gi = G.objective_gradient(vs[i])
            assert (J[i], Jd[i], Jr[i]) == (Ji, Jdi, Jri), i
            assert np.array_equal(host(gs[i]), host(gi)), i
    ws = [dev_v(d[3]) for d in data]
    vs = [dev_v(0.5 * d[2]) for d in data]
    B.set_state(vs)
    outs = B.hessian_matvec(ws)
    for i, G in enumerate(singles):
        G.objective_gradient(vs[i])
        assert np.array_equal(host(outs[i]), host(G.hessian_matvec(ws[i]))), i
    # the FP64 item against the oracle
    k = next(i for i, d in enumerate(data) if d[4] == 64)
    mT, mR, vstar, w, _ = data[k]
    c = cfgs[k]
    P = ord_.Problem(mT, mR, c["nt"], 1, c["reg"], int(c["incompressible"]), c["beta"])
    S = ord_.objective_gradient(P, 0.5 * vstar)
    J, _, _, gs = B.objective_gradient(vs)
    assert abs(J[k] - S.J) <= 1e-10 * abs(S.J)
    assert rel_inf(host(gs[k]), S.g) < 1e-10
    assert rel_inf(host(B.hessian_matvec(ws)[k]), ord_.hessian_matvec(P, S, w)) < 1e-10
    B.close()
    for G in singles:
        G.close()


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("shape,nc,gamma", [((8, 8), 1, 0), ((16, 16), 2, 1), ((32, 32), 1, 1), ((64, 64), 1, 0),
                                            ((64, 64), 3, 0)])
def test_small_grid_persistent_sweeps_equal_the_launch_path(nk, monkeypatch, shape, nc, gamma, prec):
    """Square grids up to 64^2 run the matvec's transport sweeps in one persistent
    workgroup (the recorded launches interpreted in order, workgroup barriers for kernel
    boundaries). The result equals the launch path's (NKREG_SMALL=0) and the eager
    launches' bit for bit, on the first replay and later ones, and the oracle's."""
    nt = 6
    mT, mR, vstar, w = smooth_inputs(shape, nt, nc=nc, divfree=bool(gamma))
    outs = []
    for small in ("1", "0"):
        monkeypatch.setenv("NKREG_SMALL", small)
        G = nk.Problem(shape, nt, nc=nc, reg=2, incompressible=bool(gamma), beta=1e-3, precision=prec)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        G.objective_gradient(dev_v(0.5 * vstar))
        o = G.empty_v()
        res = []
        for _ in range(3):
            G.hessian_matvec(dev_v(w), o)
            res.append(host(o))
        assert G.describe()["persistent_sweeps"] == (small == "1")
        G.use_graphs(False)
        res.append(host(G.hessian_matvec(dev_v(w))))
        outs.append(res)
        G.close()
    for r in outs[0][1:] + outs[1]:
        assert np.array_equal(outs[0][0], r)
    P = ord_.Problem(mT, mR, nt, nc, 2, gamma, 1e-3)
    S = ord_.objective_gradient(P, 0.5 * vstar)
    ref = ord_.hessian_matvec(P, S, w)
    if prec == 64:
        assert rel_inf(outs[0][0], ref) < 1e-10
    else:
        assert rel_l2(outs[0][0], ref) < 1e-5


@pytest.mark.parametrize("graphs", [True, False])
def test_batch_pcg_equals_each_items_own_pcg(nk, graphs):
    """nkreg_batch_pcg: the items (mixed grids, step counts, precisions, a checkpointed 3D
    pair) iterate in lockstep with one batched matvec per iteration; every item's x, its
    iteration count and relative residual equal its own nkreg_pcg's bit for bit, also when
    maxit stops some of them and for a zero right-hand side; with the items' graphs in use
    (each step a replayed graph, captured again for each new solution vector) and with
    direct launches."""
    probs, rhs = [], []
    for shape, nt, prec, beta, seed, ck in BATCH_ITEMS:
        gamma = len(shape) == 3
        mT, mR, vstar, w = smooth_inputs(shape, nt, divfree=gamma, seed=seed)
        G = nk.Problem(shape, nt, reg=2 if gamma else 1, incompressible=gamma, beta=beta, precision=prec,
                       checkpoint_every=ck)
        G.use_graphs(graphs)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        _, _, _, g = G.objective_gradient(dev_v(0.5 * vstar))
        probs.append(G)
        rhs.append(-g)
    rhs[3] = torch.zeros_like(rhs[3])
    B = nk.Batch(probs)
    for rtol, maxit in ((1e-6, 0), (1e-10, 3)):
        xs, its, rel, conv = B.pcg(rhs, rtol, maxit)
        for i, G in enumerate(probs):
            x, it, rr, ok = G.pcg(rhs[i], rtol, maxit)
            assert np.array_equal(host(xs[i]), host(x)), (rtol, i)
            assert its[i] == it and rel[i] == rr, (rtol, i, its[i], it, rel[i], rr)
        assert its[3] == 0 and rel[3] == 0.0
        if maxit == 3:
            assert not conv and max(its) == 3
    B.close()
    for G in probs:
        G.close()


@pytest.mark.parametrize("small", ["0", "1"])
def test_batch_items_with_different_step_counts_share_launches(nk, monkeypatch, small):
    """Items that differ only in nt form one group: each time loop runs as many iterations
    as its longest item, and the others' entries are inactive for the iterations they do
    not take. The batched gradient, the state it leaves and the batched matvec equal every
    item's own calls bit for bit, with the groups joined and with one group per step count
    (NKREG_RAGGED=0); 32^2 items also through the persistent small-grid kernel
    (NKREG_SMALL=1). Checkpointed items keep groups of their own."""
    monkeypatch.setenv("NKREG_SMALL", small)
    items = [((64, 32), 4, 32, 1e-2, 1, 0), ((64, 32), 8, 32, 1e-3, 2, 0), ((64, 32), 12, 32, 1e-2, 3, 0),
             ((32, 32), 6, 32, 1e-2, 4, 0), ((32, 32), 10, 32, 3e-2, 5, 0), ((64, 32), 8, 32, 1e-2, 6, 4),
             ((32, 32), 6, 64, 1e-2, 7, 0), ((32, 32), 4, 64, 1e-3, 8, 0)]
    cfgs, data = [], []
    for shape, nt, prec, beta, seed, ck in items:
        mT, mR, vstar, w = smooth_inputs(shape, nt, seed=seed)
        cfgs.append(dict(shape=shape, nt=nt, reg=1, beta=beta, precision=prec, checkpoint_every=ck))
        data.append((mT, mR, vstar, w, prec))
    singles = []
    for c, (mT, mR, vstar, w, prec) in zip(cfgs, data):
        G = nk.Problem(**c)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        singles.append(G)
    vs = [dev_v(0.5 * d[2]) for d in data]
    ws = [dev_v(d[3]) for d in data]
    ref_g, ref_h = [], []
    for G, v, w in zip(singles, vs, ws):
        J, Jd, Jr, g = G.objective_gradient(v)
        ref_g.append((J, Jd, Jr, host(g)))
        ref_h.append(host(G.hessian_matvec(w)))
    for ragged, sizes in (("1", [1, 2, 2, 3]), ("0", [1, 1, 1, 1, 1, 1, 1, 1])):
        monkeypatch.setenv("NKREG_RAGGED", ragged)
        B = nk.Batch.create(cfgs)
        for item, (mT, mR, vstar, w, prec) in zip(B.items, data):
            item.set_images(dev_t(mT, prec), dev_t(mR, prec))
        J, Jd, Jr, gs = B.objective_gradient(vs)
        for i in range(len(items)):
            assert (J[i], Jd[i], Jr[i]) == ref_g[i][:3], (ragged, i)
            assert np.array_equal(host(gs[i]), ref_g[i][3]), (ragged, i)
        B.set_state(vs)
        for _ in range(2):
            outs = B.hessian_matvec(ws)
            for i in range(len(items)):
                assert np.array_equal(host(outs[i]), ref_h[i]), (ragged, i)
        assert sorted(n for n, _ in B.group_plan()) == sizes, B.group_plan()
        B.close()
    for G in singles:
        G.close()


def test_small_grid_batch_groups_run_persistent(nk, monkeypatch):
    """A batch of 32^2 and 64^2 items (two persistent groups) and 128^2 items (launch
    groups): every item equals its own matvec and the launch path's bit for bit."""
    items = [((32, 32), 6, 1e-2, 1), ((32, 32), 6, 1e-3, 2), ((64, 64), 8, 1e-2, 3), ((64, 64), 8, 3e-2, 4),
             ((64, 64), 8, 1e-2, 5), ((128, 128), 8, 1e-2, 6)]
    refs = {}
    for small in ("0", "1"):
        monkeypatch.setenv("NKREG_SMALL", small)
        probs, ws = [], []
        for shape, nt, beta, seed in items:
            mT, mR, vstar, w = smooth_inputs(shape, nt, seed=seed)
            G = nk.Problem(shape, nt, reg=1, beta=beta, precision=32)
            G.set_images(dev_t(mT, 32), dev_t(mR, 32))
            G.objective_gradient(dev_v(0.5 * vstar))
            probs.append(G)
            ws.append(dev_v(w))
        singles = [host(G.hessian_matvec(wt)) for G, wt in zip(probs, ws)]
        B = nk.Batch(probs)
        for _ in range(2):
            outs = [host(o) for o in B.hessian_matvec(ws)]
            for o, r in zip(outs, singles):
                assert np.array_equal(o, r)
        refs[small] = singles
        B.close()
        for G in probs:
            G.close()
    for a, b in zip(refs["0"], refs["1"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("m,elems,lockstep", [(32, 4, 1), (128, 4, 2), (256, 4, 1), (256, 4, 2), (64, 2, 1),
                                              (64, 2, 2), (128, 2, 1), (128, 2, 2), (64, 8, 1), (256, 8, 1),
                                              (512, 8, 1)])
def test_exchange_canary_poisoned_scratch_never_reaches_the_transform(nk, m, elems, lockstep, prec):
    """The wavefront FFTs order their LDS exchanges by fences alone. With NaN written over
    the scratch before every scatter and after every gather, the forward-inverse round trip
    is NaN-free, equal to the unpoisoned run bit for bit, and m times the input."""
    import ctypes
    from paper_1408_6299_amd import _lib
    lib = _lib.load()
    count = 4099          # a ragged last wavefront
    dt = torch.float32 if prec == 32 else torch.float64
    x = torch.randn(count, m, 2, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(7))
    x = x.to(dt).contiguous()
    outs = []
    for poison in (0, 1):
        y = torch.full_like(x, float("nan"))
        st = lib.nkreg_exchange_canary(prec, m, elems, lockstep, poison, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(y.data_ptr()), count,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0, lib.nkreg_last_error().decode()
        torch.cuda.synchronize()
        outs.append(y)
    assert not torch.isnan(outs[1]).any()
    assert torch.equal(outs[0], outs[1])
    err = float(((outs[1].double() / m) - x.double()).abs().max())
    assert err < (1e-13 if prec == 64 else 1e-5), err


def test_launch_floor_chains(nk):
    """nkreg_launch_floor: graphs of dependent launches time to positive per-node costs, and
    a copy of a 512 x 256 complex spectrum costs more per node than an empty kernel."""
    t = {k: nk.launch_floor(k, 512, 256, 100) for k in nk.api.LAUNCH_FLOOR_KINDS}
    assert all(v > 0 for v in t.values()), t
    assert t["column_copy"] > t["empty"] and t["row_copy"] > t["empty"], t


def test_column_variant_pinned_per_grid(nk, monkeypatch):
    """NKREG_COL_E as grid=variant entries fixes the column pass of the grids it names and
    leaves the others to the autotuner; both variants give the same matvec bits."""
    shape, nt = (64, 64), 4
    mT, mR, vstar, w = smooth_inputs(shape, nt)
    outs = []
    for pin in ("64x64=tiled,32x32=8", "64x64=8"):
        monkeypatch.setenv("NKREG_COL_E", pin)
        G = nk.Problem(shape, nt, reg=1, beta=1e-2, precision=32)
        G.set_images(dev_t(mT, 32), dev_t(mR, 32))
        G.objective_gradient(dev_v(0.5 * vstar))
        outs.append(host(G.hessian_matvec(dev_v(w))))
        d = G.describe()
        assert d["col_E"] == (0 if "64x64=tiled" in pin else 8), d
        assert "fixed" in d["autotune"], d
        G.close()
    assert np.array_equal(outs[0], outs[1])
    monkeypatch.setenv("NKREG_COL_E", "128x128=tiled")
    G = nk.Problem((64, 32), nt, reg=1, beta=1e-2, precision=32)
    assert "fixed" not in G.describe()["autotune"]
    G.close()


@pytest.mark.parametrize("shape,nc,reg,stokes,prec", [
    ((8, 8), 1, 1, False, 64),
    ((16, 32), 2, 2, True, 32),
    ((64, 64), 3, 2, True, 32),
    ((128, 64), 1, 2, False, 64),
    ((32, 256), 1, 1, True, 64),
    ((512, 512), 1, 2, False, 32),
])
def test_fused_control_space_pass_matches_separate_passes(nk, monkeypatch, shape, nc, reg, stokes, prec):
    """On 2D grids the control-space multiplier runs as one fused column pass (k_col_spec):
    forward column transforms, the multiplier per mode (with the packed k_2 = 0 / Nyquist
    column's partner modes) and inverse transforms, across column groups of 64 columns
    (8 points) down to one (512 points). The gradient, GN matvec, P^-1, K and A agree with
    those of the separate passes (NKREG_FUSED_SPEC=0) to FP64 rounding: the lockstep
    transforms may order a butterfly's products differently, and A (|k|^4 on H2)
    amplifies a last-bit difference of the highest modes by up to (N/2)^4: the bound is
    1e-15 (N/2)^(2 reg) of the output's largest entry for A w, g and H w (which contain
    beta A), and 1e-13 for P^-1 w and K w, which amplify nothing."""
    nt = 4
    mT, mR, vstar, w = smooth_inputs(shape, nt, nc=nc, divfree=stokes)
    res = []
    for fused in (True, False):
        if fused:
            monkeypatch.delenv("NKREG_FUSED_SPEC", raising=False)
        else:
            monkeypatch.setenv("NKREG_FUSED_SPEC", "0")
        G = nk.Problem(shape, nt, nc=nc, reg=reg, incompressible=stokes, beta=1e-2, precision=prec)
        assert G.describe()["spec_fused"] is fused
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        J, _, _, g = G.objective_gradient(dev_v(0.5 * vstar))
        x = dev_v(w)
        out = [J, host(g), host(G.hessian_matvec(x)), host(G.precond(x)), host(G.project(x)), host(G.apply_reg(x))]
        res.append(out)
        G.close()
    assert abs(res[0][0] - res[1][0]) <= 1e-13 * abs(res[1][0])
    amp = (max(shape) / 2.0) ** (2 * reg)
    for name, a, b in zip(("g", "Hw", "P^-1 w", "K w", "A w"), res[0][1:], res[1][1:]):
        bound = 1e-13 if name in ("P^-1 w", "K w") else 1e-15 * amp
        assert np.max(np.abs(a - b)) <= bound * np.max(np.abs(b)), name


def test_handle_on_a_side_stream_matches_the_default_stream(nk):
    """A handle runs on the stream it was created with: work queued there (gradient,
    eager and replayed matvecs, PCG) gives the same bits as on the default stream."""
    shape, nt = (64, 32), 8
    mT, mR, vstar, w = smooth_inputs(shape, nt)
    ins = [dev_t(mT, 32), dev_t(mR, 32), dev_v(0.5 * vstar), dev_v(w)]
    res = []
    side = torch.cuda.Stream()
    for st in (torch.cuda.current_stream(), side):
        st.wait_stream(torch.cuda.current_stream())      # inputs were made on the default stream
        with torch.cuda.stream(st):
            G = nk.Problem(shape, nt, reg=2, beta=1e-3, precision=32, stream=st)
            G.set_images(ins[0], ins[1])
            J, _, _, g = G.objective_gradient(ins[2])
            outs = [G.hessian_matvec(ins[3]) for _ in range(3)]
            s, it, rel, _ = G.pcg(g, 1e-8, maxit=5)
        torch.cuda.current_stream().wait_stream(st)
        res.append([J, host(g)] + [host(o) for o in outs] + [host(s), it, rel])
        G.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_batch_items_on_two_streams(nk):
    """Items created on different streams: the batch joins every item's stream and matches
    each item's own matvec bit for bit."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    probs, ws, refs = [], [], []
    for i, (shape, nt, prec, beta, seed, ck) in enumerate(BATCH_ITEMS[:5]):
        st = side if i % 2 else torch.cuda.current_stream()
        mT, mR, vstar, w = smooth_inputs(shape, nt, seed=seed)
        ins = [dev_t(mT, prec), dev_t(mR, prec), dev_v(0.5 * vstar), dev_v(w)]
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            G = nk.Problem(shape, nt, reg=1, beta=beta, precision=prec, stream=st)
            G.set_images(ins[0], ins[1])
            G.objective_gradient(ins[2])
            refs.append(G.hessian_matvec(ins[3]))
        probs.append(G)
        ws.append(ins[3])
    torch.cuda.current_stream().wait_stream(side)
    refs = [host(r) for r in refs]
    B = nk.Batch(probs)
    outs = [p.empty_v() for p in probs]
    for _ in range(2):
        B.hessian_matvec(ws, outs)
        torch.cuda.current_stream().wait_stream(side)
        for o, r in zip(outs, refs):
            assert np.array_equal(host(o), r)
    B.close()
    for p in probs:
        p.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_newton_solve_matches_oracle(nk, prec):
    shape, nt, reg, beta = (32, 32), 8, 2, 1e-2
    P, G, _, _ = make_pair(nk, shape, nt, 1, reg, 0, beta, prec)
    v_ref, rep_ref, S_ref = okr.gauss_newton(P, gtol=1e-3, max_outer=20)
    v, rep = G.newton_solve(gtol=1e-3, max_outer=20)
    assert rep.converged and rep_ref.converged
    mis0 = np.sum((P.mR - P.mT) ** 2)
    rel_ref = 2 * S_ref.J_dist / (P.hd * mis0)
    rel_gpu = 2 * rep.J_dist / (P.hd * mis0)
    assert abs(rel_gpu - rel_ref) <= 1e-4
    if prec == 64:
        assert rep.iterations == rep_ref.iterations
        assert rel_inf(host(v), v_ref) < 1e-8
    else:
        assert abs(rep.iterations - rep_ref.iterations) <= 1
        assert rel_l2(host(v), v_ref) < 1e-3


def test_newton_history_matches_oracle_iterates(nk):
    """The per-iterate history of an FP64 solve (nkreg_solve_opts::h_history): J, ||g||_inf,
    PCG iterations and step lengths equal the oracle's at every iterate; the last row's CFL
    number and det F_1 extremes equal the oracle's at the final iterate; continuation
    appends each level's rows; the history changes no result."""
    shape, nt, reg, beta = (32, 32), 8, 2, 1e-2
    P, G, _, _ = make_pair(nk, shape, nt, 1, reg, 0, beta, 64)
    v_ref, rep_ref, _ = okr.gauss_newton(P, gtol=1e-3, max_outer=20)
    v0, rep0 = G.newton_solve(gtol=1e-3, max_outer=20)
    v, rep = G.newton_solve(gtol=1e-3, max_outer=20, history=True, history_detf=True)
    assert np.array_equal(host(v), host(v0)) and rep.iterations == rep0.iterations
    H = rep.history.numpy()
    c = {name: i for i, name in enumerate(nk.api.HISTORY_COLUMNS)}
    assert H.shape == (rep.iterations + 1, len(c))
    assert np.array_equal(H[:, c["k"]], np.arange(rep.iterations + 1))
    assert rep.iterations == rep_ref.iterations
    np.testing.assert_allclose(H[:, c["J"]], rep_ref.J, rtol=1e-9)
    np.testing.assert_allclose(H[:, c["J"]], H[:, c["J_dist"]] + H[:, c["J_reg"]], rtol=1e-14)
    np.testing.assert_allclose(H[:, c["gnorm_inf"]], rep_ref.gnorm_inf, rtol=1e-8)
    assert list(H[1:, c["cg_iterations"]].astype(int)) == list(rep_ref.cg_iterations)
    np.testing.assert_allclose(H[1:, c["alpha"]], rep_ref.alphas, rtol=0, atol=0)
    assert H[0, c["n_pde"]] == 2 and H[-1, c["n_pde"]] == rep.n_pde and np.all(np.diff(H[:, c["n_pde"]]) > 0)
    assert H[-1, c["J"]] == rep.J and H[-1, c["gnorm_inf"]] == rep.gnorm_inf
    # the final iterates agree to 1e-8 relative; CFL and det F_1 are Lipschitz in v
    assert abs(H[-1, c["cfl"]] - okr.cfl_number(v_ref, nt)) <= 1e-7 * okr.cfl_number(v_ref, nt)
    _, st_ref = odg.det_stats(v_ref, nt)
    assert abs(H[-1, c["detF_min"]] - st_ref[0]) <= 1e-7 and abs(H[-1, c["detF_max"]] - st_ref[1]) <= 1e-7
    assert H[0, c["cfl"]] == 0.0 and abs(H[0, c["detF_min"]] - 1.0) < 1e-12 and abs(H[0, c["detF_max"]] - 1.0) < 1e-12
    _, rep_nd = G.newton_solve(gtol=1e-3, max_outer=20, history=True)
    assert np.isnan(rep_nd.history.numpy()[:, 9:]).all()
    v2, reps = G.continuation([1e-1, 1e-2], gtol=1e-3, max_outer=20, history=True)
    for r in reps:
        assert tuple(r.history.shape) == (r.iterations + 1, 11) and float(r.history[-1, 1]) == r.J
    G.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_continuation_resumes_from_a_checkpoint(nk, prec, tmp_path):
    """A continuation interrupted after two of three levels, saved, loaded and resumed on a
    fresh handle, ends at the uninterrupted solve's velocity bit for bit, with the same
    iterations on the last level."""
    shape, nt, betas = (32, 32), 8, [1e-1, 1e-2, 1e-3]
    mT, mR, vstar, _ = smooth_inputs(shape, nt)

    def handle():
        G = nk.Problem(shape, nt, reg=2, beta=betas[0], precision=prec)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        return G

    G = handle()
    v_full, reps_full = G.continuation(betas, gtol=1e-3, max_outer=20)
    G.close()
    G = handle()
    v2, reps2 = G.continuation(betas[:2], gtol=1e-3, max_outer=20)
    G.close()
    path = str(tmp_path / "cont.pt")
    nk.save_continuation(path, v2, betas, 2, reps2[0].gnorm0_inf, reps2)
    G = handle()
    v3, reps3 = nk.resume_continuation(G, path, gtol=1e-3, max_outer=20)
    G.close()
    assert len(reps3) == 1 and reps3[0].iterations == reps_full[2].iterations
    assert reps3[0].cg_iterations == reps_full[2].cg_iterations
    assert np.array_equal(host(v3), host(v_full))


@pytest.mark.parametrize("prec", [64])
def test_newton_with_the_paper_stopping_rule_matches_oracle(nk, prec):
    """gtol <= 0 selects the paper's rule (C1 and C2 and C3) or C4 or C5
    (e:stopping-criteria, e:converged). FP64 library and oracle take the same outer and
    CG iterations, stop for the same reason and reach the same iterate. With a tau_J no
    solve meets, C5 (k > n_opt) ends both after n_opt + 1 iterations, unconverged."""
    shape, nt, nc, reg, gamma, beta = (32, 32), 8, 1, 2, 0, 1e-1
    P, G, _, _ = make_pair(nk, shape, nt, nc, reg, gamma, beta, prec)
    v_ref, rep_ref, _ = okr.gauss_newton(P, gtol=0.0, rule="paper", tau_J=1e-3, max_outer=50)
    v, rep = G.newton_solve(gtol=0.0, tau_J=1e-3, max_outer=50)
    assert rep_ref.converged and rep_ref.reason == "C1-C3"
    assert rep.converged and rep.stop_reason == "C1-C3"
    assert rep.iterations == rep_ref.iterations and rep.cg_iterations == rep_ref.matvecs
    assert rel_inf(host(v), v_ref) < 1e-8
    for n_opt in (0, 1):
        v_ref, rep_ref, _ = okr.gauss_newton(P, gtol=0.0, rule="paper", tau_J=1e-30, max_outer=n_opt)
        v, rep = G.newton_solve(gtol=0.0, tau_J=1e-30, max_outer=n_opt)
        assert rep_ref.reason == "C5" and not rep_ref.converged and rep_ref.iterations == n_opt + 1
        assert rep.stop_reason == "iteration limit" and not rep.converged and rep.iterations == n_opt + 1
        assert rep.cg_iterations == rep_ref.matvecs
        assert rel_inf(host(v), v_ref) < 1e-8
    G.close()


def test_warm_start_that_meets_the_relative_rule_takes_no_iteration(nk):
    """A solve started at a converged iterate with the reference gradient scale of the
    first solve (gref_inf, as continuation and the beta search pass it) stops before any
    iteration, on both sides, and reports the gradient it measured there."""
    P, G, _, _ = make_pair(nk, (32, 32), 8, 1, 2, 0, 1e-1, 64)
    v_ref, rep_ref, S_ref = okr.gauss_newton(P, gtol=1e-3, max_outer=50)
    v, rep = G.newton_solve(gtol=1e-3, max_outer=50)
    assert rep.converged and rep.iterations == rep_ref.iterations
    gref = rep_ref.gnorm0_inf
    assert abs(rep.gnorm0_inf - gref) <= 1e-10 * gref
    _, rep2_ref, S2_ref = okr.gauss_newton(P, v0=v_ref, gtol=1e-3, max_outer=50, gref_inf=gref)
    v2, rep2 = G.newton_solve(v, gtol=1e-3, max_outer=50, gref_inf=gref)
    assert rep2_ref.iterations == 0 and rep2_ref.converged
    assert rep2.iterations == 0 and rep2.converged and rep2.stop_reason == "relative gradient"
    ginf_ref = float(np.abs(S2_ref.g).max())
    assert ginf_ref <= 1e-3 * gref
    assert abs(rep2.gnorm_inf - ginf_ref) <= 1e-6 * ginf_ref
    assert np.array_equal(host(v2), host(v))
    G.close()


def test_autograd_gradient_matches_finite_differences(nk):
    from paper_1408_6299_amd import objective
    shape, nt = (32, 32), 8
    P, G, v, _ = make_pair(nk, shape, nt, 1, 2, 0, 1e-3, 64)
    vt = dev_v(v).requires_grad_(True)
    J = objective(vt, G)
    J.backward()
    grad = vt.grad.detach()
    for seed in range(20, 25):
        w = synth.bandlimited_velocity(shape, seed, 4, 0.05)
        wt = dev_v(w)
        eps = 1e-4
        jp = G.objective(dev_v(v + eps * w))[0]
        jm = G.objective(dev_v(v - eps * w))[0]
        fd = (jp - jm) / (2 * eps)
        an = float((grad * wt).sum())
        assert abs(fd - an) <= 1e-7 * abs(an) + 1e-14


@pytest.mark.parametrize("prec", [32, 64])
def test_graph_replays_match_eager_matvec(nk, prec):
    """Captured matvec graphs replayed several times, with other library work in between,
    give bit-identical results to eager launches."""
    shape, nt = (32, 64), 8
    P, G, v, w = make_pair(nk, shape, nt, 2, 2, 1, 1e-3, prec)
    G.objective_gradient(dev_v(v))
    wt = dev_v(w)
    G.use_graphs(False)
    ref = host(G.hessian_matvec(wt))
    G.use_graphs(True)
    out = G.empty_v()
    for rep in range(4):
        G.hessian_matvec(wt, out)
        assert np.array_equal(host(out), ref), rep
        G.precond(dev_v(v))                       # eager work between replays
        G.hessian_matvec(dev_v(0.5 * w))          # a different pointer pair: new capture
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("shape,nt,nc,gamma", [((32, 32), 8, 1, 0), ((8, 16, 8), 6, 2, 1)])
def test_checkpointed_trajectory_is_bit_identical(nk, shape, nt, nc, gamma, prec):
    """Keeping m every K steps and recomputing segments reproduces the full-trajectory
    gradient and matvec exactly (same kernels, same order), also when K does not divide nt.
    With S trajectory slots a sweep reuses the segments the previous sweep left in
    them, so matvecs in a row (eager, captured and replayed), a PCG solve, and a new
    gradient at another velocity followed by a matvec must all stay exact for every S,
    including S at or above the segment count."""
    mT, mR, vstar, w = smooth_inputs(shape, nt, nc=nc, divfree=bool(gamma))
    outs = []
    for K, S in ((0, 1), (3, 1), (2, 1), (2, 2), (3, 2), (2, 3), (2, 8)):
        G = nk.Problem(shape, nt, nc=nc, reg=2, incompressible=bool(gamma), beta=1e-3, precision=prec,
                       checkpoint_every=K, trajectory_slots=S)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        J, _, _, g = G.objective_gradient(dev_v(0.5 * vstar))
        res = [J, host(g), host(G.hessian_matvec(dev_v(w)))]
        wt, out = dev_v(0.3 * w + 0.1 * vstar), G.empty_v()
        for _ in range(3):                        # capture, then two replays
            G.hessian_matvec(wt, out)
            res.append(host(out))
            G.precond(dev_v(w))
        G.use_graphs(False)
        res.append(host(G.hessian_matvec(dev_v(-w))))
        G.use_graphs(True)
        s, it, rel, _ = G.pcg(g, 1e-6, maxit=6)
        res += [host(s), it, rel]
        J2, _, _, g2 = G.objective_gradient(dev_v(0.25 * vstar))
        res += [J2, host(g2), host(G.hessian_matvec(dev_v(w)))]
        outs.append(res)
        G.close()
    for res in outs[1:]:
        for a, b in zip(res, outs[0]):
            assert np.array_equal(np.asarray(a), np.asarray(b))


@pytest.mark.parametrize("prec", [32, 64])
def test_handles_of_one_grid_share_the_tile_choice(nk, prec):
    """The column-tile autotuner runs at handle creation and its choice is shared per grid
    and precision, so a second handle reproduces the first one's results bit for bit."""
    shape, nt = (64, 32), 6
    mT, mR, vstar, w = smooth_inputs(shape, nt)
    res = []
    for _ in range(2):
        G = nk.Problem(shape, nt, reg=2, beta=1e-3, precision=prec)
        desc = G.describe()
        assert desc["col_E"] in (0, 4, 8) and "col_E" in desc["autotune"], desc   # 0 = tiled
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        J, _, _, g = G.objective_gradient(dev_v(0.5 * vstar))
        res.append((desc["col_E"], J, host(g), host(G.hessian_matvec(dev_v(w)))))
        G.close()
    assert res[0][0] == res[1][0]
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][2], res[1][2])
    assert np.array_equal(res[0][3], res[1][3])


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("variant", ["8", "4", "tiled"])
@pytest.mark.parametrize("shape,nt,gamma", [((64, 128), 6, 0), ((64, 32, 64), 4, 1), ((128, 64, 32), 3, 0)])
def test_column_variants_match_oracle(nk, monkeypatch, shape, nt, gamma, variant, prec):
    """Each column-pass variant the autotuner can pick (8 or 4 complex per lane, or the
    LDS-tiled pass) gives the oracle's gradient and GN matvec, in 2D and 3D, with the tiled
    pass used on every axis long enough for it."""
    monkeypatch.setenv("NKREG_COL_E", variant)
    mT, mR, vstar, w = smooth_inputs(shape, nt, divfree=bool(gamma))
    P = ord_.Problem(mT, mR, nt, 1, 2, gamma, 1e-3)
    S = ord_.objective_gradient(P, 0.5 * vstar)
    Hw = ord_.hessian_matvec(P, S, w)
    G = nk.Problem(shape, nt, reg=2, incompressible=bool(gamma), beta=1e-3, precision=prec)
    syms = G.describe()["col_deriv_symbols"]
    if variant == "tiled":
        # axes of at least 64 points take the tiled pass, shorter ones the 8-per-lane pass
        lengths = [shape[0]] if len(shape) == 2 else [shape[1], shape[0]]
        for n_ax, sym in zip(lengths, syms):
            assert sym.startswith("k_col_t<" if n_ax >= 64 else "k_col_w<"), syms
    else:
        assert all(s.startswith("k_col_w<") and s.endswith(f", {variant}, 2>") for s in syms), syms
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    _, _, _, g = G.objective_gradient(dev_v(0.5 * vstar))
    hw = host(G.hessian_matvec(dev_v(w)))
    tol = TOL[prec]
    assert rel_l2(host(g), S.g) < (tol if prec == 64 else 1e-4)
    assert rel_l2(hw, Hw) < tol
    # spectral gradient and divergence of a smooth field go through the same passes
    u = synth.smooth_image(shape, 9, 0.6 * min(shape) ** 2 / 16.0)
    if prec == 32:
        u = u.astype(np.float32).astype(np.float64)   # the oracle sees the field the kernel sees
    gu = host(G.gradient(dev_t(u, prec)))
    assert rel_inf(gu, osp.grad(u)) < (1e-12 if prec == 64 else 2e-5)
    assert rel_l2(gu, osp.grad(u)) < (1e-12 if prec == 64 else 1e-5)
    G.close()


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("shape,nt,gamma", [((64, 128), 6, 0), ((128, 64, 64), 3, 1)])
def test_tiled_and_wave_column_passes_are_bit_identical(nk, monkeypatch, shape, nt, gamma, prec):
    """The tiled column pass and the 8-per-lane pass run the same register FFT on the same
    values, so the autotuner's choice between them never changes a result."""
    mT, mR, vstar, w = smooth_inputs(shape, nt, divfree=bool(gamma))
    outs = []
    for variant in ("8", "tiled"):
        monkeypatch.setenv("NKREG_COL_E", variant)
        G = nk.Problem(shape, nt, reg=2, incompressible=bool(gamma), beta=1e-3, precision=prec)
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        J, _, _, g = G.objective_gradient(dev_v(0.5 * vstar))
        outs.append((J, host(g), host(G.hessian_matvec(dev_v(w)))))
        G.close()
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("shape", [(256, 64, 64), (64, 256, 64)])
def test_tiled_256_point_column_pass_matches_oracle(nk, monkeypatch, shape, prec):
    """The tiled 256-point column pass (k_col_t<R, 256, CT, 2>, the pass of the 256^3
    workload) along x1 and along x2, H2 + Stokes: gradient and GN matvec at v = 0.5 v*
    against the oracle, and bit-identical to the 8-per-lane pass. FP32: the GN matvec at
    1e-5, the gradient at 1e-5 max(1, kappa / 10) of the start-of-solve gradient scale
    (lambda = m_R - m_1 amplifies the transport error by kappa), the oracle taking the
    FP32-rounded images the kernels see; FP64: 1e-10."""
    nt = 4
    mT, mR, vstar, w = smooth_inputs(shape, nt, divfree=True)
    if prec == 32:
        mT, mR = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (mT, mR))
    P = ord_.Problem(mT, mR, nt, 1, 2, 1, 1e-3)
    v = 0.5 * vstar
    S0 = ord_.objective_gradient(P, np.zeros_like(v))
    S = ord_.objective_gradient(P, v)
    Hw = ord_.hessian_matvec(P, S, w)
    outs = []
    for variant in ("tiled", "8"):
        monkeypatch.setenv("NKREG_COL_E", variant)
        G = nk.Problem(shape, nt, reg=2, incompressible=True, beta=1e-3, precision=prec)
        syms = G.describe()["col_deriv_symbols"]   # axis 1 first, then axis 0
        if variant == "tiled":
            ct = 16 if prec == 32 else 8
            long_axis = 0 if shape[0] == 256 else 1
            assert f"k_col_t<{'float' if prec == 32 else 'double'}, 256, {ct}, 2>" == syms[1 - long_axis], syms
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        J, _, _, g = G.objective_gradient(dev_v(v))
        hw = host(G.hessian_matvec(dev_v(w)))
        outs.append((J, host(g), hw))
        G.close()
    J, g, hw = outs[0]
    if prec == 64:
        assert rel_inf(g, S.g) < 1e-10 and rel_inf(hw, Hw) < 1e-10
    else:
        kappa = np.linalg.norm(P.mT) / np.linalg.norm(P.mR - P.mT)
        gscale = np.sqrt(np.sum(S0.g ** 2))
        assert np.sqrt(np.sum((g - S.g) ** 2)) < 1e-5 * max(1.0, kappa / 10.0) * gscale
        assert rel_l2(hw, Hw) < 1e-5
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])


def beta_search_problem():
    shape, nt = (16, 16), 8
    mT = synth.smooth_image(shape, 3, 0.6 * 16 ** 2 / 16)
    vstar = synth.bandlimited_velocity(shape, 77, 2, 0.5, norm="linf")
    return shape, nt, mT, otr.forward_only(mT, vstar, nt)


@pytest.mark.parametrize("prec", [64, 32])
def test_beta_search_matches_oracle(nk, prec):
    """nkreg_beta_search (decade descent, then bisection on the det F_1 bound) against the
    oracle's search: in FP64 the same trials, decisions, beta* and solution; in FP32 the
    decisions follow the bound and beta* lies within one bisection step of the oracle's."""
    shape, nt, mT, mR = beta_search_problem()
    P = ord_.Problem(mT, mR, nt, 1, 1, 0, 1.0)
    v_ref, rep_ref = okr.beta_search(P, 0.8, max_outer=10)
    G = nk.Problem(shape, nt, reg=1, beta=1.0, precision=prec)
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    v, res = G.beta_search(0.8, max_outer=10)
    assert res.breached and res.reason == "bisection converged" and res.status == 0
    for t in res.trials:
        assert (t.min_det >= 0.8) == t.accepted
    assert G.beta == res.beta_star
    if prec == 64:
        assert [t.beta for t in res.trials] == [t.beta for t in rep_ref.trials]
        assert [t.accepted for t in res.trials] == [t.accepted for t in rep_ref.trials]
        for a, b in zip(res.trials, rep_ref.trials):
            assert abs(a.min_det - b.min_det) < 1e-8 and abs(a.l2_rel - b.l2_rel) < 1e-8
        assert res.beta_star == rep_ref.beta_star and res.dbeta_min == rep_ref.dbeta_min
        assert rel_inf(host(v), v_ref) < 1e-6
    else:
        assert abs(res.beta_star - rep_ref.beta_star) <= 2 * rep_ref.dbeta_min
    _, st = G.det_grad_y(v)
    assert abs(st[0] - res.min_det_star) < 1e-12
    G.close()


def test_continuation_matches_oracle(nk):
    """nkreg_continuation: each level warm-started, every level's relative-gradient rule
    against the first level's ||g_0||_inf; FP64 against the oracle."""
    P, G, _, _ = make_pair(nk, (32, 32), 8, 1, 2, 0, 1e-1, 64)
    betas = [1e-1, 1e-2, 1e-3]
    v_ref, reps_ref = okr.continuation(P, betas)
    v, reps = G.continuation(betas)
    assert all(r.converged for r in reps)
    assert abs(reps[0].gnorm0_inf - reps_ref[0].gnorm0_inf) <= 1e-10 * reps_ref[0].gnorm0_inf
    # per level: the same outer iterations and PCG iterations as the oracle
    assert [r.iterations for r in reps] == [r.iterations for r in reps_ref]
    assert [r.cg_iterations for r in reps] == [r.matvecs for r in reps_ref]
    # The iterates agree to what the inexact solves fix, not to rounding: the last level's
    # final PCG solve runs 30 iterations at cond(P^-1 H) ~ 1e4, and FP64 CG amplifies a
    # different summation order to ~1e-5 in its output (measured 2.6e-5; a single matvec
    # and a fixed-iteration PCG solve agree to 1e-10 and 1e-9). Both final gradients meet
    # the relative rule, and the objective, stationary at the solution, agrees closely.
    assert rel_inf(host(v), v_ref) < 1e-4
    assert reps[-1].gnorm_inf <= 1e-3 * reps[0].gnorm0_inf
    # J is stationary at the solution, so it agrees to second order in the iterates'
    # distance; its data term J_dist moves to first order (measured 1.1e-4 relative)
    Pb = ord_.Problem(P.mT, P.mR, P.nt, P.nc, P.reg, P.gamma, 1e-3)
    J_ref, Jd_ref, _ = ord_.objective(Pb, v_ref)
    assert abs(reps[-1].J - J_ref) <= 1e-6 * J_ref
    assert abs(reps[-1].J_dist - Jd_ref) <= 1e-3 * Jd_ref
    assert G.beta == 1e-3


def rd_objective_dist(P, v, beta):
    Pb = ord_.Problem(P.mT, P.mR, P.nt, P.nc, P.reg, P.gamma, beta)
    return ord_.objective(Pb, v)[1]


NEWTON_CASES = [((32, 32), 8, 1, 1, 0, 1e-2), ((32, 64), 8, 3, 2, 1, 1e-3), ((16, 8, 16), 6, 1, 2, 1, 1e-3)]


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("case", NEWTON_CASES)
def test_full_newton_matvec_matches_oracle(nk, case, prec):
    """Full-Newton matvec (e:second-order-opt-cond) at a nonzero residual against the
    oracle's; it differs from the GN matvec there, and is symmetric."""
    shape, nt, nc, reg, gamma, beta = case
    P, G, v, w = make_pair(nk, shape, nt, nc, reg, gamma, beta, prec)
    G.hessian = "newton"
    S = ord_.objective_gradient(P, v)
    ref = ord_.newton_hessian_matvec(P, S, w)
    G.objective_gradient(dev_v(v))
    hw = host(G.hessian_matvec(dev_v(w)))
    # FP32: lambda = m_R - m_1 carries the cancellation error of the FP32 transport
    kappa = np.sqrt(np.sum(P.mT ** 2) / np.sum((P.mR - P.mT) ** 2))
    tol = TOL[prec] if prec == 64 else TOL[32] * max(1.0, kappa / 10.0)
    assert rel_l2(hw, ref) < tol
    gn = ord_.hessian_matvec(P, S, w)
    assert rel_l2(gn, ref) > 100 * tol
    if prec == 64:
        u = synth.bandlimited_velocity(shape, 301, 3, 0.2, divfree=bool(gamma), nc=nc)
        hu = host(G.hessian_matvec(dev_v(u)))
        a, b = float(np.sum(u * hw)), float(np.sum(hu * w))
        assert abs(a - b) <= 1e-11 * abs(a)
    G.close()


def test_full_newton_mode_errors_and_state(nk):
    """Switching the Hessian needs a new gradient."""
    shape, nt = (16, 16), 4
    mT, mR, vstar, w = smooth_inputs(shape, nt)
    G = nk.Problem(shape, nt, precision=64)
    G.set_images(dev_t(mT, 64), dev_t(mR, 64))
    G.objective_gradient(dev_v(0.5 * vstar))
    G.hessian = "newton"
    with pytest.raises(nk.NkregError) as ei:
        G.hessian_matvec(dev_v(w))
    assert ei.value.status == -5   # ESTATE
    G.objective_gradient(dev_v(0.5 * vstar))
    G.hessian_matvec(dev_v(w))
    G.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_full_newton_with_checkpointing_is_bit_identical(nk, prec):
    """The full-Newton matvec with a checkpointed state trajectory (any number of slots)
    reproduces the full-trajectory one bit for bit: matvecs in a row, a PCG solve, and a
    matvec after a new gradient."""
    shape, nt = (32, 16), 7
    mT, mR, vstar, w = smooth_inputs(shape, nt, nc=2)
    outs = []
    for K, S in ((0, 1), (2, 1), (3, 2), (2, 4)):
        G = nk.Problem(shape, nt, nc=2, reg=2, beta=1e-3, precision=prec, checkpoint_every=K, trajectory_slots=S)
        G.hessian = "newton"
        G.set_images(dev_t(mT, prec), dev_t(mR, prec))
        J, _, _, g = G.objective_gradient(dev_v(0.5 * vstar))
        res = [J, host(g)] + [host(G.hessian_matvec(dev_v(c * w))) for c in (1.0, -0.5)]
        s, it, rel, _ = G.pcg(g, 1e-6, maxit=5)
        res += [host(s), it, rel]
        G.objective_gradient(dev_v(0.25 * vstar))
        res.append(host(G.hessian_matvec(dev_v(w))))
        outs.append(res)
        G.close()
    for res in outs[1:]:
        for a, b in zip(res, outs[0]):
            assert np.array_equal(np.asarray(a), np.asarray(b))


def test_full_newton_batch_matches_single_items(nk):
    items = []
    for seed in (21, 22):
        mT, mR, vstar, w = smooth_inputs((32, 32), 6, seed=seed)
        G = nk.Problem((32, 32), 6, precision=32)
        G.hessian = "newton"
        G.set_images(dev_t(mT, 32), dev_t(mR, 32))
        G.objective_gradient(dev_v(0.5 * vstar))
        items.append((G, dev_v(w)))
    refs = [host(G.hessian_matvec(w)) for G, w in items]
    B = nk.Batch([G for G, _ in items])
    outs = B.hessian_matvec([w for _, w in items])
    assert B.groups() == [2]
    for o, r in zip(outs, refs):
        assert np.array_equal(host(o), r)


def test_pcg_negative_curvature_in_the_first_step_returns_the_preconditioned_rhs(nk):
    """Full Newton far from a minimiser (an unrelated reference image, small beta) is
    indefinite. With rhs = P u for an eigenvector u of a negative eigenvalue, the first
    search direction P^-1 rhs = u has negative curvature: PCG stops before any update
    (0 iterations, not converged) and returns P^-1 rhs, as the step length formed on the
    device leaves x untouched."""
    shape, nt, beta = (16, 16), 4, 1e-4
    width = 0.6 * 16 ** 2 / 16.0
    mT = synth.smooth_image(shape, 5, width)
    mR = synth.smooth_image(shape, 9, width)
    G = nk.Problem(shape, nt, reg=1, beta=beta, precision=64)
    G.hessian = "newton"
    G.set_images(dev_t(mT, 64), dev_t(mR, 64))
    G.objective_gradient(G.zeros_v())
    H = host(G.hessian_matrix())
    lam, U = np.linalg.eigh(0.5 * (H + H.T))
    assert lam[0] < 0, lam[:3]
    ud = dev_v(U[:, 0].reshape(G.vshape))
    assert float((ud * G.hessian_matvec(ud)).sum()) < 0
    rhs = beta * G.apply_reg(ud) + ud.mean(dim=(-2, -1), keepdim=True)   # P u, the mean kept
    pinv = host(G.precond(rhs))
    assert rel_inf(pinv, host(ud)) < 1e-8
    s, it, rel, converged = G.pcg(rhs, 1e-8)
    assert it == 0 and not converged
    assert np.array_equal(host(s), pinv)
    G.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_full_newton_solve_matches_oracle(nk, prec):
    shape, nt, reg, beta = (32, 32), 8, 2, 1e-2
    P, G, _, _ = make_pair(nk, shape, nt, 1, reg, 0, beta, prec)
    G.hessian = "newton"
    v_ref, rep_ref, S_ref = okr.gauss_newton(P, gtol=1e-3, max_outer=20, hessian="newton")
    v, rep = G.newton_solve(gtol=1e-3, max_outer=20)
    assert rep.converged and rep_ref.converged
    mis0 = np.sum((P.mR - P.mT) ** 2)
    assert abs(2 * rep.J_dist / (P.hd * mis0) - 2 * S_ref.J_dist / (P.hd * mis0)) <= 1e-4
    if prec == 64:
        assert rep.iterations == rep_ref.iterations
        assert rel_l2(host(v), v_ref) < 1e-6


@pytest.mark.parametrize("prec", [64, 32])
def test_picard_matches_oracle(nk, prec):
    """Globalised Picard iteration (preconditioned gradient descent with the step-scale
    memory) against the oracle's: FP64 the same iterations, PDE solves and iterate; FP32
    converges to the same solution."""
    mT = synth.smooth_image((16, 16), 5, 8.0)
    vstar = synth.bandlimited_velocity((16, 16), 77, 3, 0.8)
    mR = otr.forward_only(mT, vstar, 8)
    P = ord_.Problem(mT, mR, 8, 1, 1, 0, 1e-1)
    never = (0, 0.0)
    v_ref, rep_ref, _ = okr.picard(P, gtol=1e-4, max_outer=500, stagnation=(10 ** 9, 0.0))
    G = nk.Problem((16, 16), 8, reg=1, beta=1e-1, precision=prec)
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    v, rep = G.picard_solve(gtol=1e-4, max_outer=500, stagnation=never)
    assert rep.converged and rep.cg_iterations == 0
    if prec == 64:
        assert rep.iterations == rep_ref.iterations and rep.n_pde == rep_ref.n_pde
        assert rel_inf(host(v), v_ref) < 1e-8
    else:
        assert rel_l2(host(v), v_ref) < 1e-3
    _, rep_st = G.picard_solve(gtol=1e-4, max_outer=500)
    _, rep_st_ref, _ = okr.picard(P, gtol=1e-4, max_outer=500)
    if prec == 64:
        assert rep_st.iterations == rep_st_ref.iterations
    G.close()


def test_hessian_matrix_matches_oracle_columns_and_lanczos_matches_its_spectrum(nk):
    """Dense Hessian by unit-vector matvecs (16^2, n = 512) against the oracle's matvecs,
    symmetric; the Lanczos Ritz values reach its extreme eigenvalues."""
    P, G, v, _ = make_pair(nk, (16, 16), 6, 1, 2, 0, 1e-2, 64)
    S = ord_.objective_gradient(P, v)
    G.objective_gradient(dev_v(v))
    H = G.hessian_matrix()
    Hh = host(H)
    n = Hh.shape[0]
    assert n == 512
    for j in (0, 17, 300, 511):
        e = np.zeros(n)
        e[j] = 1.0
        ref = ord_.hessian_matvec(P, S, e.reshape(P.vshape())).reshape(-1)
        assert np.abs(Hh[j] - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.abs(Hh - Hh.T).max() <= 1e-12 * np.abs(Hh).max()
    ev = np.linalg.eigvalsh(0.5 * (Hh + Hh.T))
    ritz = G.lanczos(200)
    assert len(ritz) == 200
    assert abs(ritz[-1] - ev[-1]) <= 1e-10 * ev[-1]
    assert abs(ritz[0] - ev[0]) <= 1e-6 * ev[-1]
    assert ritz[0] >= ev[0] - 1e-9 * ev[-1] and ritz[-1] <= ev[-1] * (1 + 1e-12)
    G.close()


@pytest.mark.parametrize("prec,mode,K", [(32, "gn", 0), (64, "newton", 0), (32, "gn", 2)])
def test_assembled_columns_equal_single_matvecs(nk, prec, mode, K):
    """The assembly runs its unit-vector matvecs as one batch group of the handle and its
    clones (16^2: n = 512 columns, 16 replays of 32); every column equals the handle's own
    matvec of that unit vector bit for bit, also in the full-Newton mode and with a
    checkpointed trajectory."""
    nt = 6
    mT, mR, vstar, w = smooth_inputs((16, 16), nt)
    G = nk.Problem((16, 16), nt, reg=2, beta=1e-2, precision=prec, checkpoint_every=K)
    G.hessian = mode
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    G.objective_gradient(dev_v(0.5 * vstar))
    Hh = host(G.hessian_matrix())
    n = Hh.shape[0]
    assert n == 512
    for j in (0, 1, 31, 32, 257, 480, 511):
        e = np.zeros(n)
        e[j] = 1.0
        col = host(G.hessian_matvec(dev_v(e.reshape(G.vshape))))
        assert np.array_equal(Hh[j], col.reshape(-1)), j
    G.close()


GOLDEN_EIG = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "eigen_extremes.json")


def test_hessian_spectrum_extremes_match_table_t_eigenvalues(nk):
    """64^2, n_c = 1 (n = 8192), at the true velocity (zero residual): the spectrum of the
    assembled Hessian reproduces the data-independent extremes of Table t:eigenvalues.

    gamma = 0: H is symmetric; its largest eigenvalue is beta a(k) at the corner wavenumber.
    gamma = 1: H = beta A + K M (M symmetric) is not symmetric on the full space, but block
    lower-triangular in (curl-free, divergence-free) coordinates: on curl-free fields it is
    beta A (eigenvalues beta a(k), the smallest beta at |k| = 1) and on divergence-free
    fields it is the symmetric K H K. Its eigenvalues are the union of the two blocks'."""
    import json
    shape, nt = (64, 64), 8
    n = 8192
    mT = synth.smooth_image(shape, 5, 0.6 * 64 ** 2 / 16)
    k = np.fft.fftfreq(64, 1.0 / 64)
    for ent in json.load(open(GOLDEN_EIG))["entries"]:
        gamma, reg, beta = ent["gamma"], ent["reg"], ent["beta"]
        vstar = synth.bandlimited_velocity(shape, 77, 4, synth.cfl_literal_linf(64, nt), divfree=bool(gamma),
                                           norm="linf")
        mR = otr.forward_only(mT, vstar, nt)
        G = nk.Problem(shape, nt, reg=reg, incompressible=bool(gamma), beta=beta, precision=64)
        G.set_images(dev_t(mT, 64), dev_t(mR, 64))
        G.objective_gradient(dev_v(vstar))
        H = G.hessian_matrix()
        assert H.shape == (n, n)
        if not gamma:
            assert float((H - H.T).abs().max()) <= 1e-12 * float(H.abs().max())
            ev = torch.linalg.eigvalsh(0.5 * (H + H.T)).cpu().numpy()
            lo, hi = ev[0], ev[-1]
        else:
            # divergence-free block: K H K with K assembled column by column by nkreg_project
            Km = torch.empty((n, n), dtype=torch.float64, device="cuda")
            e = G.zeros_v()
            for j in range(n):
                e.view(-1).zero_()
                e.view(-1)[j] = 1.0
                Km[j] = G.project(e).view(-1)
            Hd = Km @ H.T @ Km      # rows of H are H e_j, so H.T is the operator's matrix
            evd = torch.linalg.eigvalsh(0.5 * (Hd + Hd.T)).cpu().numpy()
            rank = n - int(round(float(torch.trace(Km))))      # curl-free dimension
            evd = evd[rank:]                                    # drop the curl-free null directions
            # curl-free block: beta a(k) on the curl-free Fourier modes (k != 0)
            kk = k[:, None] ** 2 + k[None, :] ** 2
            a = (kk if reg == 1 else kk ** 2)[kk > 0]
            lo, hi = min(evd[0], beta * a.min()), max(evd[-1], beta * a.max())
            # the curl-free block is exactly beta A: (I - K) H w = beta A w for w = grad cos(x1)
            x1 = 2 * np.pi * np.arange(64) / 64
            w = np.zeros(G.vshape)
            w[0, 0] = -np.sin(x1)[:, None] * np.ones(64)[None, :]
            Hw = host(G.hessian_matvec(dev_v(w)))
            cf = Hw - host(G.project(dev_v(Hw)))
            assert np.abs(cf - beta * w).max() <= 1e-9 * beta
            del Km, Hd
        if "max_real" in ent:
            assert abs(hi - ent["max_real"]) <= 1e-9 * ent["max_real"], (ent, hi)
        if "min_real" in ent:
            assert abs(lo - ent["min_real"]) <= 1e-9 * ent["min_real"], (ent, lo)
        assert lo > 0
        del H
        G.close()


EDGE_SHAPES = [((8, 8), 1, 1, 1, 0), ((512, 8), 3, 1, 2, 0), ((8, 512), 3, 2, 1, 1),
               ((512, 8, 8), 2, 1, 2, 1), ((8, 512, 8), 2, 1, 1, 0), ((8, 8, 512), 2, 1, 2, 0),
               ((8, 8, 8), 1, 2, 1, 1)]


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("shape,nt,nc,reg,gamma", EDGE_SHAPES)
def test_extreme_shapes_match_oracle(nk, shape, nt, nc, reg, gamma, prec):
    """Smallest (8) and largest (512) axis lengths on every axis position, one time step,
    several Chebyshev coefficients: gradient and GN matvec against the oracle.

    On a 512-point axis the H2 symbol reaches 256^4, so the problem itself amplifies FP64
    rounding: the FP64 bound is 20 times the oracle's own change under a 1e-16 relative
    perturbation of v (and of w for the matvec), at least 1e-10. FP32 (FFTs of length 512, CFL-0.1 steps with only
    one to three time steps) is held to 3e-5 here."""
    mT, mR, vstar, w = smooth_inputs(shape, max(nt, 2), nc=nc, divfree=bool(gamma))
    mR = otr.forward_only(mT, vstar, nt)
    P = ord_.Problem(mT, mR, nt, nc, reg, gamma, 1e-2)
    v = 0.5 * vstar
    S = ord_.objective_gradient(P, v)
    Hw = ord_.hessian_matvec(P, S, w)
    G = nk.Problem(shape, nt, nc=nc, reg=reg, incompressible=bool(gamma), beta=1e-2, precision=prec)
    G.set_images(dev_t(mT, prec), dev_t(mR, prec))
    J, _, _, g = G.objective_gradient(dev_v(v))
    hw = host(G.hessian_matvec(dev_v(w)))
    if prec == 64:
        rng = np.random.default_rng(0)
        vp = v * (1 + 1e-16 * rng.standard_normal(v.shape))
        Sp = ord_.objective_gradient(P, vp)
        sens_g = rel_inf(Sp.g, S.g)
        wp = w * (1 + 1e-16 * rng.standard_normal(w.shape))
        sens_h = rel_inf(ord_.hessian_matvec(P, Sp, wp), Hw)
        assert abs(J - S.J) <= 1e-10 * abs(S.J)
        assert rel_inf(host(g), S.g) < max(1e-10, 20 * sens_g)
        assert rel_inf(hw, Hw) < max(1e-10, 20 * sens_h)
    else:
        kappa = np.sqrt(np.sum(P.mT ** 2) / max(np.sum((P.mR - P.mT) ** 2), 1e-300))
        assert rel_l2(host(g), S.g) < 3e-5 * max(1.0, kappa / 10.0)
        assert rel_l2(hw, Hw) < 3e-5
    G.close()
