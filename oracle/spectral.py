"""Fourier pseudospectral operators on the periodic box (FP64, CPU).

Paper: Section "Numerical Discretization" (spectral derivatives, h_x = 2 pi / n_x),
Section "Inversion: Regularization Operators" (spectral inverse of beta A with the
base frequency set to one), Section "Elimination of p and p~" (equation
e:eliminated-control: K[f] = f - grad(Lap^-1(div f))), and equations
e:first-variation-H1 (A = -Lap) and e:first-variation-H2 (A = Lap^2).

Readings where the paper is silent:
* Wavenumbers are the integers k_i in {-N_i/2, .., N_i/2 - 1}.
* First derivatives multiply by i*k_i with the Nyquist wavenumber k_i = -N_i/2
  set to zero. That makes the discrete derivative a real skew matrix, so the
  conservative adjoint transport is the exact transpose of the state transport.
* Even-order symbols keep the Nyquist wavenumber: |k|^2 = sum k_i^2. The
  paper's Table t:eigenvalues (largest eigenvalue at beta = 1e6 on 64^2 equal to
  1e6 * (32^2 + 32^2)^2 for H2 and 1e6 * (32^2 + 32^2) for H1) fixes this.
* K uses the Nyquist-zeroed wavevector, so div(K f) vanishes for the discrete
  divergence above; K is the identity where that wavevector is zero.
* The preconditioner divides by beta * a(k) for k != 0 and leaves k = 0 alone.

Fields are NumPy arrays with the spatial axes last; axis -d is x1.
The complex FFT over all spatial axes is used throughout (plain, not fast).
"""
from __future__ import annotations

import os
from functools import lru_cache
from typing import Sequence, Tuple

import numpy as np
import scipy.fft as sfft

WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", os.cpu_count() or 1))


def set_workers(n: int) -> None:
    global WORKERS
    WORKERS = max(1, int(n))


def fft(u: np.ndarray, d: int) -> np.ndarray:
    """Forward DFT over the last d axes: u_hat(k) = sum_x u(x) exp(-i k.x)."""
    return sfft.fftn(u, axes=tuple(range(-d, 0)), workers=WORKERS)


def ifft_real(uh: np.ndarray, d: int) -> np.ndarray:
    """Inverse DFT over the last d axes, keeping the real part."""
    return sfft.ifftn(uh, axes=tuple(range(-d, 0)), workers=WORKERS).real


@lru_cache(maxsize=64)
def wavenumbers(shape: Tuple[int, ...]) -> Tuple[np.ndarray, ...]:
    """Integer wavenumbers k_i (FFT ordering), broadcastable over ``shape``."""
    d = len(shape)
    out = []
    for i, n in enumerate(shape):
        k = np.fft.fftfreq(n, 1.0 / n)
        s = [1] * d
        s[i] = n
        out.append(k.reshape(s))
    return tuple(out)


@lru_cache(maxsize=64)
def first_derivative_symbols(shape: Tuple[int, ...]) -> Tuple[np.ndarray, ...]:
    """i * k_i with the Nyquist wavenumber k_i = -N_i/2 set to zero."""
    out = []
    for n, k in zip(shape, wavenumbers(shape)):
        kk = np.where(k == -(n // 2), 0.0, k)
        out.append(1j * kk)
    return tuple(out)


@lru_cache(maxsize=64)
def ksq(shape: Tuple[int, ...]) -> np.ndarray:
    """|k|^2 = sum_i k_i^2, Nyquist kept (symbol of -Lap)."""
    ks = wavenumbers(shape)
    return sum(k * k for k in ks)


def reg_symbol(shape: Tuple[int, ...], reg: int) -> np.ndarray:
    """Symbol a(k) of A: |k|^2 for H1 (A = -Lap), |k|^4 for H2 (A = Lap^2)."""
    if reg not in (1, 2):
        raise ValueError("reg must be 1 (H1) or 2 (H2)")
    return ksq(shape) ** reg


def grad(u: np.ndarray) -> np.ndarray:
    """Spectral gradient of a scalar field u (shape = grid); returns (d, *grid)."""
    d = u.ndim
    uh = fft(u, d)
    return np.stack([ifft_real(s * uh, d) for s in first_derivative_symbols(u.shape)])


def div(w: np.ndarray) -> np.ndarray:
    """Spectral divergence sum_i D_i w^i of a vector field w (shape (d, *grid))."""
    d = w.shape[0]
    shape = w.shape[1:]
    syms = first_derivative_symbols(shape)
    acc = np.zeros(shape, dtype=np.complex128)
    for i in range(d):
        acc += syms[i] * fft(w[i], d)
    return ifft_real(acc, d)


def apply_A(v: np.ndarray, reg: int, d: int) -> np.ndarray:
    """A applied per component to fields whose last d axes are the grid.

    A = -Lap (H1) or Lap^2 (H2), i.e. multiplication of each Fourier mode by
    a(k) = |k|^2 or |k|^4 (e:first-variation-H1, e:first-variation-H2).
    """
    a = reg_symbol(v.shape[-d:], reg)
    return ifft_real(a * fft(v, d), d)


def apply_K(f: np.ndarray) -> np.ndarray:
    """K[f] = f - grad(Lap^-1 div f) for one vector field f of shape (d, *grid).

    Computed per Fourier mode as (I - kt kt^T / |kt|^2) f_hat with kt the
    Nyquist-zeroed wavevector (identity where kt = 0).
    """
    d = f.shape[0]
    shape = f.shape[1:]
    syms = first_derivative_symbols(shape)
    kt = [s.imag for s in syms]
    kt2 = sum(k * k for k in kt)
    safe = np.where(kt2 > 0, kt2, 1.0)
    fh = np.stack([fft(f[i], d) for i in range(d)])
    proj = sum(kt[i] * fh[i] for i in range(d)) / safe
    proj = np.where(kt2 > 0, proj, 0.0)
    return np.stack([ifft_real(fh[i] - kt[i] * proj, d) for i in range(d)])


def apply_Pinv(r: np.ndarray, reg: int, beta: float, d: int) -> np.ndarray:
    """Preconditioner (beta A)^-1 on fields whose last d axes are the grid.

    Each mode is divided by beta * a(k); the k = 0 mode, which A annihilates,
    gets the factor 1 instead (Section "Inversion: Regularization Operators").
    """
    a = reg_symbol(r.shape[-d:], reg)
    den = np.where(a > 0, beta * a, 1.0)
    return ifft_real(fft(r, d) / den, d)


def inner_h(a: np.ndarray, b: np.ndarray, shape: Sequence[int]) -> float:
    """Discrete L2 inner product <a, b>_h = h_d * sum a*b, h_d = prod(2 pi / N_i)."""
    hd = float(np.prod([2.0 * np.pi / n for n in shape]))
    return hd * float(np.sum(a * b))


def cell_volume(shape: Sequence[int]) -> float:
    return float(np.prod([2.0 * np.pi / n for n in shape]))
