"""Pins of the oracle's Heun transport solves (state, adjoint, incremental).

Closed forms (constant velocity), exact invariants (constant images, mass of
the conservative adjoint), the exact-shift convergence order and the
transpose identity between the forward and the adjoint solve.
"""
import numpy as np
import pytest

from oracle import spectral as sp
from oracle import transport as tr
import synth


def small_velocity(shape, nc=1, seed=21, kmax=3, target=0.8, divfree=False):
    return synth.bandlimited_velocity(shape, seed, kmax, target, divfree=divfree, nc=nc)


def test_constant_image_is_transported_unchanged():
    shape = (16, 16)
    v = small_velocity(shape, nc=2)
    m = np.full(shape, 0.37)
    m1 = tr.forward_only(m, v, 8)
    assert np.abs(m1 - 0.37).max() < 1e-14


@pytest.mark.parametrize("shape", [(16, 16), (8, 8, 8)])
def test_constant_velocity_closed_form(shape):
    """Heun with constant c: m_hat_1(k) = G(-i h c.kt)^nt m_hat_T(k), G(z) = 1 + z + z^2/2."""
    d = len(shape)
    c = np.array([0.7, -0.4, 0.25][:d])
    v = np.zeros((1, d) + shape)
    for i in range(d):
        v[0, i] = c[i]
    mT = synth.smooth_image(shape, 4, 6.0)
    nt = 7
    h = 1.0 / nt
    m1 = tr.forward_only(mT, v, nt)
    kt = [s.imag for s in sp.first_derivative_symbols(shape)]
    z = -1j * h * sum(c[i] * kt[i] for i in range(d))
    G = 1 + z + z * z / 2
    ref = np.fft.ifftn(G ** nt * np.fft.fftn(mT)).real
    assert np.abs(m1 - ref).max() < 1e-13


def test_exact_shift_error_is_second_order():
    shape = (32, 32)
    x1, x2 = synth.grid_coords(shape)
    c = (0.9, -0.6)
    mT = np.sin(x1) * np.cos(2 * x2) + 0.3 * np.cos(3 * x1)
    exact = np.sin(x1 - c[0]) * np.cos(2 * (x2 - c[1])) + 0.3 * np.cos(3 * (x1 - c[0]))
    v = np.zeros((1, 2) + shape)
    v[0, 0], v[0, 1] = c
    errs = [np.abs(tr.forward_only(mT, v, nt) - exact).max() for nt in (8, 16, 32)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.6 < r < 4.4 for r in ratios), (errs, ratios)


def test_adjoint_conserves_mass():
    shape = (16, 16)
    v = small_velocity(shape, nc=2, divfree=False)
    rng = np.random.default_rng(1)
    lam1 = rng.standard_normal(shape)
    traj = tr.forward_state(np.zeros(shape), v, 6)
    lam0, _ = tr.adjoint_with_force(lam1, v, traj, 6)
    assert abs(lam0.sum() - lam1.sum()) < 1e-11


@pytest.mark.parametrize("nc", [1, 2, 3])
def test_adjoint_solve_is_the_transpose_of_the_forward_solve(nc):
    """<Psi mu, a> = <mu, Phi a>: Phi = m_T -> m_1 (linear for fixed v), Psi = lam_1 -> lam_0."""
    shape = (8, 8)
    nt = 5
    v = small_velocity(shape, nc=nc, target=1.1)
    rng = np.random.default_rng(2)
    a = rng.standard_normal(shape)
    mu = rng.standard_normal(shape)
    Phi_a = tr.forward_only(a, v, nt)
    traj = tr.forward_state(np.zeros(shape), v, nt)
    Psi_mu, _ = tr.adjoint_with_force(mu, v, traj, nt)
    lhs, rhs = np.sum(Psi_mu * a), np.sum(mu * Phi_a)
    assert abs(lhs - rhs) <= 1e-14 * np.sqrt(np.sum(a * a) * np.sum(mu * mu)) * 10


def test_forward_state_and_forward_only_agree():
    shape = (16, 16)
    v = small_velocity(shape, nc=2)
    mT = synth.smooth_image(shape, 3, 8.0)
    a = tr.forward_only(mT, v, 6)
    b = tr.forward_state(mT, v, 6).m1
    assert np.abs(a - b).max() == 0.0


def test_incremental_state_is_the_directional_derivative_of_the_forward_solve():
    """m~_1 = d/de m_1(v + e w) at e = 0, by central differences (O(e^2))."""
    shape = (16, 16)
    nt = 6
    v = small_velocity(shape, nc=2)
    w = small_velocity(shape, nc=2, seed=33, target=0.5)
    mT = synth.smooth_image(shape, 3, 8.0)
    traj = tr.forward_state(mT, v, nt)
    mt = tr.incremental_state(v, w, traj, nt)
    errs = []
    for eps in (1e-2, 1e-3):
        fd = (tr.forward_only(mT, v + eps * w, nt) - tr.forward_only(mT, v - eps * w, nt)) / (2 * eps)
        errs.append(np.abs(fd - mt).max() / np.abs(mt).max())
    assert errs[1] < 1e-6
    assert errs[0] / errs[1] > 50
