"""Seeded synthetic inputs for the registration problem (images and velocities).

This module is shared by the FP64 oracle, the tests and the benchmark. It
holds no arithmetic of the registration method itself: it only draws seeded
random Fourier coefficients and synthesises real fields from them with
``numpy.fft.irfftn``. Everything the method computes (transport, gradients,
projections, regularisation) lives elsewhere.

The paper's images (the "sinusoidal", "UT", hand and brain images of its
numerical study) are not available, so smooth random fields with the same
sizes (64^2 .. 512^2) and the same intensity range [0, 1] stand in for them.

Grid convention (same as the method's): x_j = 2*pi*j/N_i, j = 0..N_i-1, on
the periodic box [0, 2*pi)^d; axis 0 is x1 and the last axis is contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "grid_coords", "integer_wavenumbers", "smooth_image", "bandlimited_velocity",
    "c0_velocity", "chebyshev_sample_max", "ProblemSpec", "CONFIGS", "make_inputs", "cfl_steps",
    "batch_specs_nteff",
    "batch_specs", "cfl_literal_linf",
]


def grid_coords(shape: Sequence[int]) -> List[np.ndarray]:
    """Nodal coordinates x_i = 2*pi*j/N_i broadcast to the full grid (axis 0 = x1)."""
    axes = [2.0 * np.pi * np.arange(n) / n for n in shape]
    return list(np.meshgrid(*axes, indexing="ij"))


def integer_wavenumbers(shape: Sequence[int], half_last: bool = True) -> List[np.ndarray]:
    """Integer wavenumber grids matching numpy's (r)fftn layouts, broadcastable."""
    d = len(shape)
    out = []
    for i, n in enumerate(shape):
        if half_last and i == d - 1:
            k = np.arange(n // 2 + 1, dtype=np.float64)
        else:
            k = np.fft.fftfreq(n, 1.0 / n)
        s = [1] * d
        s[i] = k.size
        out.append(k.reshape(s))
    return out


def _random_half_spectrum(rng: np.random.Generator, shape: Sequence[int]) -> np.ndarray:
    hshape = list(shape[:-1]) + [shape[-1] // 2 + 1]
    re = rng.standard_normal(hshape)
    im = rng.standard_normal(hshape)
    return re + 1j * im


def smooth_image(shape: Sequence[int], seed: int, width: float) -> np.ndarray:
    """Smooth random image in [0, 1].

    Half-spectrum coefficients (xi1 + i*xi2) * exp(-|k|^2 / width), xi ~ N(0,1)
    from ``numpy.random.default_rng(seed)``, synthesised with irfftn and
    min-max normalised to [0, 1].
    """
    rng = np.random.default_rng(seed)
    c = _random_half_spectrum(rng, shape)
    ks = integer_wavenumbers(shape)
    k2 = sum(k * k for k in ks)
    c = c * np.exp(-k2 / width)
    m = np.fft.irfftn(c, s=tuple(shape), axes=tuple(range(len(shape))))
    m = (m - m.min()) / (m.max() - m.min())
    return np.ascontiguousarray(m, dtype=np.float64)


def _field_from_half(c: np.ndarray, shape: Sequence[int]) -> np.ndarray:
    return np.fft.irfftn(c, s=tuple(shape), axes=tuple(range(len(shape))))


def _raw_bandlimited(rng: np.random.Generator, shape: Sequence[int], kmax: float,
                     divfree: bool) -> np.ndarray:
    """One random band-limited vector field (not yet scaled), shape (d, *shape).

    Per component, coefficients xi * (1 + |k|^2)^-2 on 0 < |k|_2 <= kmax. A
    divergence-free field is synthesised as a curl: in 2D v = (d2 psi, -d1 psi)
    from a random stream function psi, in 3D v = curl(psi) from a random vector
    potential; the potential's coefficients carry an extra 1/|k| so that v keeps
    the (1 + |k|^2)^-2 envelope.
    """
    d = len(shape)
    ks = integer_wavenumbers(shape)
    k2 = sum(k * k for k in ks)
    band = (k2 > 0) & (k2 <= kmax * kmax)
    env = np.where(band, 1.0 / (1.0 + k2) ** 2, 0.0)
    if not divfree:
        comps = []
        for _ in range(d):
            c = _random_half_spectrum(rng, shape) * env
            comps.append(_field_from_half(c, shape))
        return np.stack(comps)
    kabs = np.sqrt(np.where(k2 > 0, k2, 1.0))
    if d == 2:
        psi = _random_half_spectrum(rng, shape) * env / kabs
        v1 = _field_from_half(1j * ks[1] * psi, shape)
        v2 = _field_from_half(-1j * ks[0] * psi, shape)
        return np.stack([v1, v2])
    psi = [_random_half_spectrum(rng, shape) * env / kabs for _ in range(3)]
    k1, k2_, k3 = ks
    w1 = 1j * (k2_ * psi[2] - k3 * psi[1])
    w2 = 1j * (k3 * psi[0] - k1 * psi[2])
    w3 = 1j * (k1 * psi[1] - k2_ * psi[0])
    return np.stack([_field_from_half(w, shape) for w in (w1, w2, w3)])


def chebyshev_sample_max(vl: np.ndarray, nsamples: int = 65) -> float:
    """max over x and over t in {0, 1/(ns-1), .., 1} of |sum_l T_{l-1}(2t-1) v_l(x)|_2."""
    nc = vl.shape[0]
    best = 0.0
    for t in np.linspace(0.0, 1.0, nsamples):
        coef = [np.polynomial.chebyshev.chebval(2.0 * t - 1.0, np.eye(nc)[l]) for l in range(nc)]
        v = sum(c * vl[l] for l, c in enumerate(coef))
        best = max(best, float(np.sqrt((v * v).sum(axis=0)).max()))
    return best


def bandlimited_velocity(shape: Sequence[int], seed: int, kmax: float, target: float,
                         divfree: bool = False, nc: int = 1, norm: str = "l2") -> np.ndarray:
    """Random band-limited velocity coefficients v_l, shape (nc, d, *shape).

    Scaled so that the maximum over x (and over sampled t for nc > 1) of the
    pointwise Euclidean norm (``norm="l2"``) or of the largest component
    magnitude (``norm="linf"``) equals ``target``.
    """
    rng = np.random.default_rng(seed)
    vl = np.stack([_raw_bandlimited(rng, shape, kmax, divfree) for _ in range(nc)])
    if norm == "l2":
        cur = chebyshev_sample_max(vl)
    elif norm == "linf":
        cur = float(np.abs(vl).max()) if nc == 1 else _linf_sample_max(vl)
    else:
        raise ValueError(norm)
    return np.ascontiguousarray(vl * (target / cur), dtype=np.float64)


def _linf_sample_max(vl: np.ndarray, nsamples: int = 65) -> float:
    nc = vl.shape[0]
    best = 0.0
    for t in np.linspace(0.0, 1.0, nsamples):
        coef = [np.polynomial.chebyshev.chebval(2.0 * t - 1.0, np.eye(nc)[l]) for l in range(nc)]
        v = sum(c * vl[l] for l, c in enumerate(coef))
        best = max(best, float(np.abs(v).max()))
    return best


def c0_velocity(shape: Sequence[int], amplitude: float = 1.0) -> np.ndarray:
    """The 64^2 configuration's stationary velocity, shape (1, 2, N1, N2).

    v = a * (0.5 sin x2 cos x1, 0.5 cos x2 sin x1). It is the gradient of
    0.5 a sin x1 sin x2, hence curl-free and compressible.
    """
    if len(shape) != 2:
        raise ValueError("c0_velocity is two-dimensional")
    x1, x2 = grid_coords(shape)
    v = np.stack([0.5 * np.sin(x2) * np.cos(x1), 0.5 * np.cos(x2) * np.sin(x1)])
    return np.ascontiguousarray(amplitude * v[None], dtype=np.float64)


def cfl_literal_linf(n: int, nt: int, cfl: float = 0.1) -> float:
    """Largest component magnitude that keeps h_t * max|v^i| / h_x^i at ``cfl``."""
    return cfl * 2.0 * np.pi * nt / n


@dataclass
class ProblemSpec:
    """Everything that defines one registration problem instance."""
    name: str
    shape: Tuple[int, ...]
    nt: int
    nc: int
    reg: int            # 1: H1 seminorm (A = -Lap), 2: H2 seminorm (A = Lap^2)
    gamma: int          # 1: incompressible (Leray projection of the body force)
    beta: float
    precision: int      # working precision of the fields: 32 or 64
    image_seed: int
    image_width: float
    vel_kind: str       # "c0" | "band"
    vel_seed: int = 0
    vel_kmax: float = 0.0
    vel_target: float = 1.0
    vel_norm: str = "l2"
    vel_divfree: bool = False
    vel_amplitude: float = 1.0
    beta_levels: Tuple[float, ...] = ()
    checkpoint_every: int = 0
    extra: Dict[str, object] = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return len(self.shape)


def _spec_table() -> Dict[str, ProblemSpec]:
    c = {}
    c["c0"] = ProblemSpec("c0: 2D 64x64 FP64, H1 beta=1e-2, nt=16", (64, 64), 16, 1, 1, 0, 1e-2,
                          64, 0, 36.0, "c0")
    c["c1"] = ProblemSpec("c1: 2D 256x256, 3 Chebyshev coefficients, H2 + Stokes, beta=1e-3, nt=408",
                          (256, 256), 408, 3, 2, 1, 1e-3, 32, 1, 400.0, "band", vel_seed=101,
                          vel_kmax=8, vel_target=1.0, vel_norm="l2", vel_divfree=True)
    c["c2"] = ProblemSpec("c2: 2D 512x512 FP32, H2 beta continuation 1e-1..1e-4, nt=1224",
                          (512, 512), 1224, 1, 2, 0, 1e-4, 32, 2, 400.0, "band", vel_seed=102,
                          vel_kmax=16, vel_target=1.5, vel_norm="l2",
                          beta_levels=(1e-1, 1e-2, 1e-3, 1e-4))
    c["c2lit"] = ProblemSpec("c2lit: 2D 512x512 FP32, H2, nt=32 (velocity scaled to CFL 0.1)",
                             (512, 512), 32, 1, 2, 0, 1e-4, 32, 2, 400.0, "band", vel_seed=102,
                             vel_kmax=16, vel_target=cfl_literal_linf(512, 32), vel_norm="linf",
                             beta_levels=(1e-1, 1e-2, 1e-3, 1e-4))
    c["c2beta"] = ProblemSpec("c2beta: 2D 256x256, H1, nt=64 (CFL 0.095), beta search with eps_F = 0.85",
                              (256, 256), 64, 1, 1, 0, 1.0, 32, 2, 400.0, "band", vel_seed=211, vel_kmax=4,
                              vel_target=0.15, vel_norm="linf", extra={"eps_F": 0.85})
    c["c4"] = ProblemSpec("c4: 3D 256^3 FP32, H2 + Stokes, beta=1e-3, nt=32 (CFL 0.1), checkpoint 8",
                          (256, 256, 256), 32, 1, 2, 1, 1e-3, 32, 4, 256.0, "band", vel_seed=104,
                          vel_kmax=8, vel_target=cfl_literal_linf(256, 32), vel_norm="linf",
                          vel_divfree=True, checkpoint_every=8)
    return c


CONFIGS: Dict[str, ProblemSpec] = _spec_table()


def make_velocity(spec: ProblemSpec) -> np.ndarray:
    if spec.vel_kind == "c0":
        return c0_velocity(spec.shape, spec.vel_amplitude)
    return bandlimited_velocity(spec.shape, spec.vel_seed, spec.vel_kmax, spec.vel_target,
                                spec.vel_divfree, spec.nc, spec.vel_norm)


def make_inputs(spec: ProblemSpec) -> Tuple[np.ndarray, np.ndarray]:
    """Template image m_T and true velocity coefficients v* (FP64, host)."""
    mT = smooth_image(spec.shape, spec.image_seed, spec.image_width)
    return mT, make_velocity(spec)


def batch_specs(count: int = 64, seed: int = 3, nt: int = 16,
                sizes: Sequence[int] = (64, 128, 256, 512)) -> List[ProblemSpec]:
    """The batched workload: independent 2D pairs of uneven grid sizes.

    Grid sizes are drawn uniformly from ``sizes`` and amplitudes a_i from
    U[0.5, 1.5] with ``default_rng(seed)``; item i uses image seed 1000+i and
    the 64^2 configuration's velocity scaled by a_i * s_N, where s_N puts the
    largest amplitude (a = 1.5) at CFL 0.1 for ``nt`` steps on an N^2 grid.
    """
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    amps = rng.uniform(0.5, 1.5, size=count)
    out = []
    for i in range(count):
        n = int(ns[i])
        s_n = cfl_literal_linf(n, nt) / (0.5 * 1.5)
        out.append(ProblemSpec(f"batch item {i}: {n}x{n}", (n, n), nt, 1, 1, 0, 1e-2, 32,
                               1000 + i, 36.0, "c0", vel_amplitude=float(amps[i] * s_n)))
    return out


def cfl_steps(vmax_linf: float, n: int, cfl: float = 0.1, multiple: int = 8, nt_min: int = 16) -> int:
    """Time steps that keep h_t * max|v^i| / h_x at or below ``cfl`` on an n-point axis,
    at least ``nt_min`` and rounded up to a multiple of ``multiple``."""
    nt = int(np.ceil(vmax_linf * n / (2.0 * np.pi * cfl)))
    nt = max(nt_min, nt)
    return -(-nt // multiple) * multiple


def batch_specs_nteff(count: int = 64, seed: int = 3, cfl: float = 0.1, multiple: int = 64,
                      sizes: Sequence[int] = (64, 128, 256, 512)) -> List[ProblemSpec]:
    """The batched workload at its own amplitudes: the grid sizes and amplitudes of
    batch_specs (same draws), each item's velocity the 64^2 configuration's scaled by a_i
    (max|v^i| = a_i / 2), and each item's steps set by the CFL bound at ``cfl`` (rounded up
    to a multiple of ``multiple``, so items of one grid share a few step counts)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    amps = rng.uniform(0.5, 1.5, size=count)
    out = []
    for i in range(count):
        n = int(ns[i])
        a = float(amps[i])
        nt = cfl_steps(0.5 * a, n, cfl, multiple)
        out.append(ProblemSpec(f"batch item {i}: {n}x{n}, nt {nt}", (n, n), nt, 1, 1, 0, 1e-2, 32,
                               1000 + i, 36.0, "c0", vel_amplitude=a))
    return out
