"""Pins of the oracle's spectral operators against brute force, closed forms and the paper.

Nothing here calls the GPU library.
"""
import json
import os

import numpy as np
import pytest

from oracle import spectral as sp
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_dft_derivative(u, axis):
    """D_axis u by explicit O(N^2d) DFT sums (no FFT library): the textbook
    trigonometric interpolant differentiated, with the Nyquist wavenumber dropped."""
    shape = u.shape
    d = u.ndim
    xs = [2 * np.pi * np.arange(n) / n for n in shape]
    ks = [np.array([k if k < n // 2 else k - n for k in range(n)], dtype=float) for n in shape]
    X = np.stack(np.meshgrid(*xs, indexing="ij")).reshape(d, -1)          # (d, P)
    K = np.stack(np.meshgrid(*ks, indexing="ij")).reshape(d, -1)          # (d, P)
    E = np.exp(-1j * (K.T @ X))                                           # E[k, x]
    uh = E @ u.reshape(-1)
    n_ax = shape[axis]
    kk = K[axis].copy()
    kk[kk == -(n_ax // 2)] = 0.0
    out = (np.conj(E).T @ (1j * kk * uh)) / u.size
    return out.real.reshape(shape), np.abs(out.imag).max()


@pytest.mark.parametrize("shape", [(8, 8), (8, 16), (4, 8, 8)])
def test_grad_matches_brute_force_dft(shape):
    rng = np.random.default_rng(11)
    u = rng.standard_normal(shape)
    g = sp.grad(u)
    for ax in range(len(shape)):
        ref, imag = brute_dft_derivative(u, ax)
        assert imag < 1e-12
        assert np.abs(g[ax] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_derivative_of_trig_polynomial_is_exact():
    x1, x2 = synth.grid_coords((32, 16))
    u = np.sin(3 * x1) * np.cos(2 * x2)
    g = sp.grad(u)
    assert np.abs(g[0] - 3 * np.cos(3 * x1) * np.cos(2 * x2)).max() < 1e-12
    assert np.abs(g[1] + 2 * np.sin(3 * x1) * np.sin(2 * x2)).max() < 1e-12
    w = np.stack([np.sin(x1), np.cos(5 * x2)])
    assert np.abs(sp.div(w) - (np.cos(x1) - 5 * np.sin(5 * x2))).max() < 1e-12


def test_derivative_3d_trig():
    x1, x2, x3 = synth.grid_coords((8, 16, 8))
    u = np.cos(x1) * np.sin(3 * x2) * np.cos(2 * x3)
    g = sp.grad(u)
    assert np.abs(g[0] + np.sin(x1) * np.sin(3 * x2) * np.cos(2 * x3)).max() < 1e-12
    assert np.abs(g[1] - 3 * np.cos(x1) * np.cos(3 * x2) * np.cos(2 * x3)).max() < 1e-12
    assert np.abs(g[2] + 2 * np.cos(x1) * np.sin(3 * x2) * np.sin(2 * x3)).max() < 1e-12


def test_nyquist_mode_has_zero_first_derivative():
    # cos(N/2 x) sampled on the grid is (-1)^j; its derivative -N/2 sin(N/2 x) vanishes there.
    x1, x2 = synth.grid_coords((16, 16))
    u = np.cos(8 * x1) + np.cos(8 * x2)
    assert np.abs(sp.grad(u)).max() < 1e-12


def dense(op, shape):
    n = int(np.prod(shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(op(e.reshape(shape)).reshape(-1))
    return np.stack(cols, axis=1)


def test_first_derivative_is_real_skew():
    for ax in range(2):
        D = dense(lambda u: sp.grad(u)[ax], (8, 8))
        assert np.abs(D + D.T).max() < 1e-13


def test_divergence_is_minus_transpose_of_gradient():
    shape = (8, 8)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(shape)
    w = rng.standard_normal((2,) + shape)
    lhs = np.sum(sp.div(w) * u)
    rhs = -np.sum(w * sp.grad(u))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_K_is_an_orthogonal_projection_onto_divergence_free_fields():
    shape = (8, 8)
    n = int(np.prod(shape))
    Kd = dense(lambda f: sp.apply_K(f), (2,) + shape)
    assert np.abs(Kd @ Kd - Kd).max() < 1e-13
    assert np.abs(Kd - Kd.T).max() < 1e-13
    rng = np.random.default_rng(5)
    f = rng.standard_normal((2,) + shape)
    assert np.abs(sp.div(sp.apply_K(f))).max() < 1e-12
    # gradients are removed, curls are kept (analytic fields)
    x1, x2 = synth.grid_coords((16, 16))
    phi_grad = np.stack([np.cos(x1) * np.cos(2 * x2), -2 * np.sin(x1) * np.sin(2 * x2)])
    assert np.abs(sp.apply_K(phi_grad)).max() < 1e-12
    curl = np.stack([2 * np.sin(x1) * np.cos(2 * x2), -np.cos(x1) * np.sin(2 * x2)])
    assert np.abs(sp.apply_K(curl) - curl).max() < 1e-12
    # constants pass through
    c = np.ones((2,) + (16, 16)) * np.array([0.3, -0.7])[:, None, None]
    assert np.abs(sp.apply_K(c) - c).max() < 1e-14


def test_K_removes_config0_velocity():
    # The 64^2 configuration's velocity is the gradient of 0.5 sin x1 sin x2.
    v = synth.c0_velocity((64, 64))[0]
    assert np.abs(sp.apply_K(v)).max() < 1e-12
    assert np.abs(sp.div(v)).max() > 0.9


@pytest.mark.parametrize("reg", [1, 2])
def test_A_on_trig_polynomials(reg):
    x1, x2 = synth.grid_coords((32, 32))
    u = np.sin(3 * x1) * np.cos(2 * x2)
    Au = sp.apply_A(u[None], reg, 2)[0]
    assert np.abs(Au - (13.0 ** reg) * u).max() < 1e-9 * 13.0 ** reg


def test_A_keeps_the_nyquist_wavenumber_and_matches_paper_extremes():
    with open(os.path.join(GOLDEN, "eigen_extremes.json")) as fh:
        gold = json.load(fh)
    shape = tuple(gold["grid"])
    j1, j2 = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    corner = (-1.0) ** (j1 + j2)
    for e in gold["entries"]:
        if "max_real" not in e:
            continue
        Au = sp.apply_A(corner[None], e["reg"], 2)[0]
        lam = e["beta"] * float(np.sum(Au * corner) / np.sum(corner * corner))
        assert lam == pytest.approx(e["max_real"], rel=1e-12)


@pytest.mark.parametrize("reg", [1, 2])
def test_preconditioner_inverts_beta_A_on_mean_free_fields(reg):
    rng = np.random.default_rng(7)
    u = rng.standard_normal((2, 16, 16))
    u -= u.mean(axis=(1, 2), keepdims=True)
    beta = 3e-3
    back = sp.apply_Pinv(beta * sp.apply_A(u, reg, 2), reg, beta, 2)
    assert np.abs(back - u).max() < 1e-10
    c = np.full((2, 16, 16), 0.25)
    assert np.abs(sp.apply_Pinv(c, reg, beta, 2) - c).max() < 1e-14


def test_fft_parseval_and_hermitian():
    rng = np.random.default_rng(9)
    u = rng.standard_normal((16, 8))
    uh = sp.fft(u, 2)
    assert abs(np.sum(np.abs(uh) ** 2) / u.size - np.sum(u * u)) < 1e-10
    n1, n2 = u.shape
    for k1 in range(n1):
        for k2 in range(n2):
            assert abs(uh[k1, k2] - np.conj(uh[(-k1) % n1, (-k2) % n2])) < 1e-12
