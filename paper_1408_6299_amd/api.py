"""Python face of the gfx950 registration library.

Thin wrapper over the C ABI (include/nkreg.h): it checks and marshals torch
tensors (device memory) and passes torch's current HIP stream. Every step of
the computation runs in the library's HIP kernels; nothing here computes.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_int, c_void_p
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import Config, NkregError, SolveOpts, SolveReport, check

__all__ = ["Problem", "Batch", "NkregError", "SolveResult"]


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


@dataclass
class SolveResult:
    iterations: int
    cg_iterations: int
    n_pde: int
    line_search_failed: bool
    converged: bool
    J0: float
    J: float
    J_dist: float
    J_reg: float
    gnorm0_inf: float
    gnorm_inf: float
    seconds: float
    status: int
    stop_reason: str = ""
    # one row per iterate v_k (k = 0, 1, ...), columns HISTORY_COLUMNS (min and max det F_1
    # are NaN unless det F was asked for), as a float64 host tensor; None unless asked for
    history: Optional[torch.Tensor] = None


HISTORY_COLUMNS = ("k", "J", "J_dist", "J_reg", "gnorm_inf", "cg_iterations", "alpha", "n_pde", "cfl", "detF_min",
                   "detF_max")

STOP_REASONS = {1: "relative gradient", 2: "C1-C3", 3: "C4", 4: "iteration limit", 5: "line search failed",
                6: "objective stagnation"}


@dataclass
class BetaTrial:
    beta: float
    min_det: float
    l2_rel: float
    accepted: bool


BETA_SEARCH_REASONS = {1: "bisection converged", 2: "L2 distance stagnates", 3: "lower bound on beta",
                       4: "step limit", 5: "bound breached at the first beta"}


@dataclass
class BetaSearchResult:
    trials: List[BetaTrial]
    beta_star: float
    min_det_star: float
    l2_rel_star: float
    dbeta_min: float
    breached: bool
    reason: str
    newton_iterations: int
    cg_iterations: int
    seconds: float
    status: int

    @property
    def steps(self) -> int:
        return len(self.trials)


class Problem:
    """One registration problem (images, grid, time steps, regulariser) on the current GPU.

    Tensors live on the GPU and are contiguous. Images and other scalar fields
    have shape ``shape`` and the transport dtype: float32 (``precision=32``) or
    float64 (``precision=64``). Velocity-shaped arrays (velocity coefficients,
    gradients, Hessian products, Krylov vectors) have shape (nc, d, *shape) and
    are float64 in both modes.

    ``checkpoint_every=K`` keeps the state every K steps instead of the whole
    trajectory of gradients; ``trajectory_slots=S`` keeps S K-step segments of
    that trajectory, so a Hessian matvec recomputes 2 (ceil(nt/K) - S) segments.
    Neither changes any result.
    """

    def __init__(self, shape: Sequence[int], nt: int, nc: int = 1, reg: int = 1,
                 incompressible: bool = False, beta: float = 1e-2, precision: int = 32,
                 cfl_max: float = 0.0, stream: Optional[torch.cuda.Stream] = None,
                 checkpoint_every: int = 0, trajectory_slots: int = 1):
        cfg = self._setup(shape, nt, nc, reg, incompressible, beta, precision, cfl_max, stream, checkpoint_every,
                          trajectory_slots)
        h = c_void_p()
        check(self.lib.nkreg_create(byref(cfg), c_void_p(self.stream.cuda_stream), byref(h)), "nkreg_create")
        self._h = h
        self._owned = True

    def _setup(self, shape, nt, nc, reg, incompressible, beta, precision, cfl_max, stream, checkpoint_every,
               trajectory_slots) -> Config:
        """Records the configuration on the object and returns it as the C struct."""
        self.lib = _lib.load()
        self.shape = tuple(int(s) for s in shape)
        self.d = len(self.shape)
        self.nt, self.nc, self.reg = int(nt), int(nc), int(reg)
        self.incompressible = bool(incompressible)
        self.precision = int(precision)
        self.dtype = torch.float32 if self.precision == 32 else torch.float64
        self.vdtype = torch.float64
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = Config()
        cfg.dim = self.d
        for i in range(3):
            cfg.n[i] = self.shape[i] if i < self.d else 1
        cfg.nt, cfg.nc, cfg.reg = self.nt, self.nc, self.reg
        cfg.incompressible = int(self.incompressible)
        cfg.beta = float(beta)
        cfg.precision = self.precision
        cfg.checkpoint_every = int(checkpoint_every)
        cfg.trajectory_slots = int(trajectory_slots)
        cfg.cfl_max = float(cfl_max)
        self._beta = float(beta)
        return cfg

    @classmethod
    def _borrowed(cls, handle: c_void_p, **kw) -> "Problem":
        """A view of a handle owned elsewhere (a batch's item); closing it does nothing."""
        p = cls.__new__(cls)
        p._setup(**kw)
        p._h = handle
        p._owned = False
        return p

    # -- lifetime --
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            if getattr(self, "_owned", True):
                self.lib.nkreg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --
    @property
    def vshape(self) -> Tuple[int, ...]:
        return (self.nc, self.d) + self.shape

    @property
    def hd(self) -> float:
        import math
        out = 1.0
        for n in self.shape:
            out *= 2.0 * math.pi / n
        return out

    @property
    def beta(self) -> float:
        return self._beta

    @beta.setter
    def beta(self, value: float) -> None:
        check(self.lib.nkreg_set_beta(self._h, c_double(value)), "nkreg_set_beta")
        self._beta = float(value)

    @property
    def hessian(self) -> str:
        """"gn" (Gauss-Newton, default) or "newton" (full Newton, e:second-order-opt-cond)."""
        return getattr(self, "_hessian", "gn")

    @hessian.setter
    def hessian(self, mode: str) -> None:
        if mode not in ("gn", "newton"):
            raise ValueError("hessian must be 'gn' or 'newton'")
        check(self.lib.nkreg_set_hessian(self._h, c_int(1 if mode == "newton" else 0)), "nkreg_set_hessian")
        self._hessian = mode

    def hessian_matrix(self) -> torch.Tensor:
        """The dense Hessian at the cached state, (n, n) float64 with n = nc*d*prod(shape);
        row j is H e_j (n matvecs)."""
        nvals = self.nc * self.d * int(torch.tensor(self.shape).prod())
        H = torch.empty((nvals, nvals), dtype=torch.float64, device=self.device)
        check(self.lib.nkreg_hessian_assemble(self._h, _ptr(H)), "nkreg_hessian_assemble")
        return H

    def lanczos(self, steps: int = 100) -> List[float]:
        """Ritz values (ascending) of up to ``steps`` Lanczos steps on the Hessian."""
        ritz = (c_double * max(1, steps))()
        cnt = c_int()
        check(self.lib.nkreg_hessian_lanczos(self._h, c_int(steps), ritz, byref(cnt)), "nkreg_hessian_lanczos")
        return [ritz[i] for i in range(cnt.value)]

    def describe(self) -> dict:
        """Launch configuration of the handle (tile choices, autotuner timings)."""
        import json
        buf = ctypes.create_string_buffer(8192)
        check(self.lib.nkreg_describe(self._h, buf, 8192), "nkreg_describe")
        return json.loads(buf.value.decode())

    def use_graphs(self, enable: bool) -> None:
        """Replay Hessian matvecs (and a batch item's PCG step) from captured HIP graphs
        (default) or launch eagerly."""
        check(self.lib.nkreg_use_graphs(self._h, c_int(int(enable))), "nkreg_use_graphs")

    def _check(self, t: torch.Tensor, shape: Tuple[int, ...], name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must live on the GPU")
        want = self.vdtype if tuple(shape) == self.vshape else self.dtype
        if t.dtype != want:
            raise TypeError(f"{name} has dtype {t.dtype}, expected {want}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def empty_v(self) -> torch.Tensor:
        return torch.empty(self.vshape, dtype=self.vdtype, device=self.device)

    def zeros_v(self) -> torch.Tensor:
        return torch.zeros(self.vshape, dtype=self.vdtype, device=self.device)

    # -- the calls of the C ABI --
    def set_images(self, mT: torch.Tensor, mR: torch.Tensor) -> None:
        self._check(mT, self.shape, "mT")
        self._check(mR, self.shape, "mR")
        check(self.lib.nkreg_set_images(self._h, _ptr(mT), _ptr(mR)), "nkreg_set_images")

    def forward(self, v: torch.Tensor) -> torch.Tensor:
        self._check(v, self.vshape, "v")
        m1 = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        check(self.lib.nkreg_forward(self._h, _ptr(v), _ptr(m1)), "nkreg_forward")
        return m1

    def objective(self, v: torch.Tensor) -> Tuple[float, float, float]:
        self._check(v, self.vshape, "v")
        J, Jd, Jr = c_double(), c_double(), c_double()
        check(self.lib.nkreg_objective(self._h, _ptr(v), byref(J), byref(Jd), byref(Jr)), "nkreg_objective")
        return J.value, Jd.value, Jr.value

    def objective_gradient(self, v: torch.Tensor, g: Optional[torch.Tensor] = None):
        self._check(v, self.vshape, "v")
        if g is None:
            g = self.empty_v()
        self._check(g, self.vshape, "g")
        J, Jd, Jr = c_double(), c_double(), c_double()
        check(self.lib.nkreg_objective_gradient(self._h, _ptr(v), byref(J), byref(Jd), byref(Jr), _ptr(g)),
              "nkreg_objective_gradient")
        return J.value, Jd.value, Jr.value, g

    def hessian_matvec(self, vt: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check(vt, self.vshape, "vt")
        if out is None:
            out = self.empty_v()
        self._check(out, self.vshape, "out")
        check(self.lib.nkreg_hessian_matvec(self._h, _ptr(vt), _ptr(out)), "nkreg_hessian_matvec")
        return out

    def precond(self, r: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check(r, self.vshape, "r")
        out = self.empty_v() if out is None else out
        check(self.lib.nkreg_precond_apply(self._h, _ptr(r), _ptr(out)), "nkreg_precond_apply")
        return out

    def project(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check(f, self.vshape, "f")
        out = self.empty_v() if out is None else out
        check(self.lib.nkreg_project(self._h, _ptr(f), _ptr(out)), "nkreg_project")
        return out

    def apply_reg(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check(x, self.vshape, "x")
        out = self.empty_v() if out is None else out
        check(self.lib.nkreg_apply_reg(self._h, _ptr(x), _ptr(out)), "nkreg_apply_reg")
        return out

    def pcg(self, rhs: torch.Tensor, rtol: float, maxit: int = 0, out: Optional[torch.Tensor] = None):
        """Returns (s, iterations, relative residual, converged)."""
        self._check(rhs, self.vshape, "rhs")
        out = self.empty_v() if out is None else out
        it, rr = c_int(), c_double()
        st = self.lib.nkreg_pcg(self._h, _ptr(rhs), _ptr(out), c_double(rtol), c_int(maxit), byref(it), byref(rr))
        if st not in (_lib.OK, _lib.ENOCONV):
            check(st, "nkreg_pcg")
        return out, it.value, rr.value, st == _lib.OK

    def det_grad_y(self, v: torch.Tensor) -> Tuple[torch.Tensor, Tuple[float, float, float, float]]:
        self._check(v, self.vshape, "v")
        det = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        stats = (c_double * 4)()
        check(self.lib.nkreg_det_grad_y(self._h, _ptr(v), _ptr(det), stats), "nkreg_det_grad_y")
        return det, tuple(stats)

    def newton_solve(self, v: Optional[torch.Tensor] = None, gtol: float = 1e-3, max_outer: int = 50,
                     tau_J: float = 1e-3, pcg_maxit: int = 0, cfl_guard: bool = False,
                     verbose: bool = False, gref_inf: float = 0.0, history: bool = False,
                     history_detf: bool = False) -> Tuple[torch.Tensor, SolveResult]:
        """Gauss-Newton-Krylov solve from v (zero if None); returns (v, report).

        ``gref_inf`` > 0 replaces ||g_0||_inf in the relative gradient rule (used by
        beta continuation to measure every level against the first level's gradient).
        ``history`` returns one row per iterate (HISTORY_COLUMNS) in the report;
        ``history_detf`` adds det F_1's extremes at every iterate (one FP64 solve each).
        """
        v = self.zeros_v() if v is None else v.clone()
        self._check(v, self.vshape, "v")
        o = self._solve_opts(gtol, max_outer, tau_J, pcg_maxit, cfl_guard, verbose, gref_inf,
                             history_rows=max_outer + 2 if history else 0, history_detf=history_detf)
        rep = SolveReport()
        st = self.lib.nkreg_newton_solve(self._h, _ptr(v), byref(o), byref(rep))
        if st not in (_lib.OK, _lib.ENOCONV):
            check(st, "nkreg_newton_solve")
        return v, self._result(rep, st, o)

    @staticmethod
    def _solve_opts(gtol=1e-3, max_outer=50, tau_J=1e-3, pcg_maxit=0, cfl_guard=False, verbose=False,
                    gref_inf=0.0, history_rows=0, history_detf=False) -> SolveOpts:
        o = SolveOpts()
        o.max_outer, o.gtol, o.tau_J = int(max_outer), float(gtol), float(tau_J)
        o.pcg_maxit, o.cfl_guard, o.verbose = int(pcg_maxit), int(cfl_guard), int(verbose)
        o.gref_inf = float(gref_inf)
        o.history_detf = int(history_detf)
        if history_rows > 0:
            buf = (c_double * (history_rows * _lib.HISTORY_COLS))()
            o.h_history = ctypes.cast(buf, ctypes.POINTER(c_double))
            o.history_cap = int(history_rows)
            o._history_buf = buf          # keeps the array alive with the options
        return o

    @staticmethod
    def _history(o: SolveOpts, first: int, rows: int) -> Optional[torch.Tensor]:
        buf = getattr(o, "_history_buf", None)
        if buf is None:
            return None
        c = _lib.HISTORY_COLS
        return torch.tensor(buf[first * c:(first + rows) * c], dtype=torch.float64).view(rows, c)

    @staticmethod
    def _result(rep: SolveReport, st: int, o: Optional[SolveOpts] = None, first: int = 0) -> "SolveResult":
        hist = None if o is None else Problem._history(o, first, rep.history_rows)
        return SolveResult(rep.iterations, rep.cg_iterations, rep.n_pde, bool(rep.line_search_failed),
                           bool(rep.converged), rep.J0, rep.J, rep.J_dist, rep.J_reg, rep.gnorm0_inf,
                           rep.gnorm_inf, rep.seconds, st, STOP_REASONS.get(rep.stop_reason, ""), hist)

    def picard_solve(self, v: Optional[torch.Tensor] = None, gtol: float = 1e-3, max_outer: int = 500,
                     memory: bool = True, stagnation: Tuple[int, float] = (10, 1e-6), **kw
                     ) -> Tuple[torch.Tensor, SolveResult]:
        """Globalised Picard iteration (preconditioned gradient descent with the step-scale
        memory) from v (zero if None); returns (v, report). stagnation = (count, tol),
        count <= 0 disables the objective-stagnation stop."""
        v = self.zeros_v() if v is None else v.clone()
        self._check(v, self.vshape, "v")
        history = kw.pop("history", False)
        o = self._solve_opts(gtol=gtol, max_outer=max_outer, history_rows=max_outer + 2 if history else 0, **kw)
        po = _lib.PicardOpts()
        po.memory, po.stagnation_count, po.stagnation_tol = int(memory), int(stagnation[0]), float(stagnation[1])
        rep = SolveReport()
        st = self.lib.nkreg_picard_solve(self._h, _ptr(v), byref(o), byref(po), byref(rep))
        if st not in (_lib.OK, _lib.ENOCONV):
            check(st, "nkreg_picard_solve")
        return v, self._result(rep, st, o)

    def continuation(self, betas: Sequence[float], v: Optional[torch.Tensor] = None, gtol: float = 1e-3,
                     max_outer: int = 50, **kw) -> Tuple[torch.Tensor, list]:
        """Solve for each beta in turn, warm-starting from the previous level; the relative
        gradient rule of every level is measured against the first level's ||g_0||_inf
        (nkreg_continuation). Returns (v, one report per level)."""
        v = self.zeros_v() if v is None else v.clone()
        self._check(v, self.vshape, "v")
        n = len(betas)
        bs = (c_double * max(1, n))(*[float(b) for b in betas])
        reps = (SolveReport * max(1, n))()
        history = kw.pop("history", False)
        o = self._solve_opts(gtol=gtol, max_outer=max_outer,
                             history_rows=n * (max_outer + 2) if history else 0, **kw)
        st = self.lib.nkreg_continuation(self._h, _ptr(v), bs, n, byref(o), reps)
        if st not in (_lib.OK, _lib.ENOCONV):
            check(st, "nkreg_continuation")
        if n:
            self._beta = float(betas[-1])
        out, first = [], 0
        for i in range(n):
            out.append(self._result(reps[i], st, o, first))
            first += reps[i].history_rows
        return v, out

    def beta_search(self, eps_F: float, v: Optional[torch.Tensor] = None, beta_start: float = 1.0,
                    beta_min: float = 1e-6, dbeta_rel: float = 0.05, l2_rel_min: float = 1e-2,
                    max_steps: int = 0, gtol: float = 1e-3, max_outer: int = 50, **kw
                    ) -> Tuple[torch.Tensor, "BetaSearchResult"]:
        """Parameter continuation in beta with the lower bound eps_F on det F_1
        (nkreg_beta_search); returns (solution at beta*, result with every trial)."""
        v = self.zeros_v() if v is None else v.clone()
        self._check(v, self.vshape, "v")
        o = _lib.BetaSearchOpts()
        o.eps_F, o.beta_start, o.beta_min = float(eps_F), float(beta_start), float(beta_min)
        o.dbeta_rel, o.l2_rel_min, o.max_steps = float(dbeta_rel), float(l2_rel_min), int(max_steps)
        o.solve = self._solve_opts(gtol=gtol, max_outer=max_outer, **kw)
        r = _lib.BetaSearchReport()
        st = self.lib.nkreg_beta_search(self._h, _ptr(v), byref(o), byref(r))
        if st not in (_lib.OK, _lib.ENOCONV):
            check(st, "nkreg_beta_search")
        if r.steps and r.beta_star == r.beta_star:
            self._beta = float(r.beta_star)
        trials = [BetaTrial(r.trial_beta[i], r.trial_min_det[i], r.trial_l2_rel[i], bool(r.trial_accepted[i]))
                  for i in range(r.steps)]
        res = BetaSearchResult(trials, r.beta_star, r.min_det_star, r.l2_rel_star, r.dbeta_min, bool(r.breached),
                               BETA_SEARCH_REASONS.get(r.reason, str(r.reason)), r.newton_iterations,
                               r.cg_iterations, r.seconds, st)
        return v, res

    def gradient(self, u: torch.Tensor) -> torch.Tensor:
        self._check(u, self.shape, "u")
        out = torch.empty((self.d,) + self.shape, dtype=self.dtype, device=self.device)
        check(self.lib.nkreg_gradient(self._h, _ptr(u), _ptr(out)), "nkreg_gradient")
        return out

    def divergence(self, w: torch.Tensor) -> torch.Tensor:
        self._check(w, (self.d,) + self.shape, "w")
        out = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        check(self.lib.nkreg_divergence(self._h, _ptr(w), _ptr(out)), "nkreg_divergence")
        return out

    # kernel identifiers for timer_arm
    KERNELS = {"state1": 0, "state2": 1, "inc1": 2, "inc2": 3, "adjinit": 4, "adj1": 5, "adj2": 6,
               "r2c": 7, "c2r": 8, "grad": 9, "div": 10, "col_fwd": 20, "col_inv": 21, "col_deriv": 22}

    def timer_arm(self, kernel: str, capacity: int = 4096) -> None:
        """Time each of the next ``capacity`` launches of ``kernel`` with dispatch-stamped HIP events."""
        check(self.lib.nkreg_timer_arm(self._h, c_int(self.KERNELS[kernel]), c_int(capacity)), "nkreg_timer_arm")

    def matvec_bytes(self, vt: torch.Tensor) -> Tuple[float, int]:
        """(algorithmic bytes, launches) of one Hessian matvec at the cached state."""
        self._check(vt, self.vshape, "vt")
        out = self.empty_v()
        b, n = c_double(), c_int()
        check(self.lib.nkreg_matvec_bytes(self._h, _ptr(vt), _ptr(out), byref(b), byref(n)), "nkreg_matvec_bytes")
        return b.value, n.value

    def timer_read(self) -> Tuple[int, float, float]:
        """(launches, average ms per launch, algorithmic bytes per launch); disarms."""
        n, ms, b = c_int(), c_double(), c_double()
        check(self.lib.nkreg_timer_read(self._h, byref(n), byref(ms), byref(b)), "nkreg_timer_read")
        return n.value, ms.value, b.value

    def dot(self, a: torch.Tensor, b: torch.Tensor) -> float:
        """FP64 inner product sum(a*b) of two float64 GPU tensors of equal size."""
        if a.dtype != torch.float64 or b.dtype != torch.float64 or a.numel() != b.numel():
            raise ValueError("dot: operands must be float64 tensors of equal size")
        out = c_double()
        check(self.lib.nkreg_dot(self._h, _ptr(a.contiguous()), _ptr(b.contiguous()), a.numel(), byref(out)),
              "nkreg_dot")
        return out.value


LAUNCH_FLOOR_KINDS = {"empty": 0, "row_copy": 1, "column_copy": 2, "row_column_alternating": 3}


def launch_floor(kind: str, rows: int = 512, cols: int = 256, nodes: int = 200) -> float:
    """Microseconds per node of a graph of dependent launches over a rows x cols complex
    FP32 array (nkreg_launch_floor): "empty", "row_copy", "column_copy" or
    "row_column_alternating"; runs on torch's current stream."""
    lib = _lib.load()
    us = c_double()
    check(lib.nkreg_launch_floor(LAUNCH_FLOOR_KINDS[kind], int(rows), int(cols), int(nodes),
                                 c_void_p(torch.cuda.current_stream().cuda_stream), byref(us)), "nkreg_launch_floor")
    return us.value


class Batch:
    """Several independent problems whose gradients and Hessian matvecs are applied in one
    call each (one HIP-graph launch over all items; items of one configuration share every
    kernel launch).

    ``Batch(problems)`` batches existing problems (which stay owned by the caller);
    ``Batch.create(configs)`` makes the problems itself (``items`` gives them; they are
    destroyed with the batch).
    """

    def __init__(self, problems: Sequence[Problem]):
        self.lib = _lib.load()
        self.problems = list(problems)
        arr = (c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        h = c_void_p()
        check(self.lib.nkreg_batch_wrap(len(self.problems), arr, byref(h)), "nkreg_batch_wrap")
        self._h = h

    @classmethod
    def create(cls, configs: Sequence[dict], stream: Optional[torch.cuda.Stream] = None) -> "Batch":
        """configs: keyword dicts of Problem (shape, nt, nc, reg, incompressible, beta,
        precision, cfl_max, checkpoint_every, trajectory_slots)."""
        b = cls.__new__(cls)
        b.lib = _lib.load()
        st = stream if stream is not None else torch.cuda.current_stream()
        defaults = dict(nc=1, reg=1, incompressible=False, beta=1e-2, precision=32, cfl_max=0.0,
                        checkpoint_every=0, trajectory_slots=1)
        kws, cfgs = [], (Config * max(1, len(configs)))()
        for i, c in enumerate(configs):
            kw = dict(defaults, **c)
            kw["stream"] = st
            tmp = Problem.__new__(Problem)
            cfgs[i] = tmp._setup(**kw)
            kws.append(kw)
        h = c_void_p()
        check(b.lib.nkreg_batch_create(len(configs), cfgs, c_void_p(st.cuda_stream), byref(h)), "nkreg_batch_create")
        b._h = h
        b.problems = []
        for i, kw in enumerate(kws):
            ih = c_void_p()
            check(b.lib.nkreg_batch_item(h, i, byref(ih)), "nkreg_batch_item")
            b.problems.append(Problem._borrowed(ih, **kw))
        return b

    @property
    def items(self) -> List[Problem]:
        return self.problems

    def objective_gradient(self, vs: Sequence[torch.Tensor], gs: Optional[Sequence[torch.Tensor]] = None):
        """Every item's objective and gradient at vs[i]; returns (J, J_dist, J_reg, gs)."""
        n = len(self.problems)
        if gs is None:
            gs = [p.empty_v() for p in self.problems]
        for p, a, b in zip(self.problems, vs, gs):
            p._check(a, p.vshape, "v")
            p._check(b, p.vshape, "g")
        ins = (c_void_p * n)(*[t.data_ptr() for t in vs])
        os_ = (c_void_p * n)(*[t.data_ptr() for t in gs])
        J, Jd, Jr = (c_double * n)(), (c_double * n)(), (c_double * n)()
        check(self.lib.nkreg_batch_objective_gradient(self._h, ins, J, Jd, Jr, os_), "nkreg_batch_objective_gradient")
        return list(J), list(Jd), list(Jr), gs

    def pcg(self, rhs: Sequence[torch.Tensor], rtol: float, maxit: int = 0,
            outs: Optional[Sequence[torch.Tensor]] = None):
        """PCG on every item at its cached state, all items iterating in lockstep with one
        batched matvec per iteration (nkreg_batch_pcg). Returns (xs, iterations, relative
        residuals, all converged); each item's results equal its own Problem.pcg's."""
        n = len(self.problems)
        outs = [p.empty_v() for p in self.problems] if outs is None else list(outs)
        for p, a, b in zip(self.problems, rhs, outs):
            p._check(a, p.vshape, "rhs")
            p._check(b, p.vshape, "x")
        ins = (c_void_p * n)(*[t.data_ptr() for t in rhs])
        os_ = (c_void_p * n)(*[t.data_ptr() for t in outs])
        its, rel = (c_int * n)(), (c_double * n)()
        st = self.lib.nkreg_batch_pcg(self._h, ins, os_, c_double(rtol), c_int(maxit), its, rel)
        if st not in (_lib.OK, _lib.ENOCONV):
            check(st, "nkreg_batch_pcg")
        return outs, list(its), list(rel), st == _lib.OK

    def set_state(self, vs: Sequence[torch.Tensor]) -> None:
        """Every item's forward and adjoint sweeps at vs[i] (the state its matvecs use)."""
        n = len(self.problems)
        for p, a in zip(self.problems, vs):
            p._check(a, p.vshape, "v")
        ins = (c_void_p * n)(*[t.data_ptr() for t in vs])
        check(self.lib.nkreg_batch_set_state(self._h, ins), "nkreg_batch_set_state")

    def hessian_matvec(self, vts: Sequence[torch.Tensor], outs: Optional[Sequence[torch.Tensor]] = None):
        if outs is None:
            outs = [p.empty_v() for p in self.problems]
        for p, a, b in zip(self.problems, vts, outs):
            p._check(a, p.vshape, "vt")
            p._check(b, p.vshape, "out")
        n = len(self.problems)
        ins = (c_void_p * n)(*[t.data_ptr() for t in vts])
        os_ = (c_void_p * n)(*[t.data_ptr() for t in outs])
        check(self.lib.nkreg_batch_hessian_matvec(self._h, ins, os_), "nkreg_batch_hessian_matvec")
        return outs

    def groups(self) -> List[int]:
        """Sizes of the item groups that share launches in the last built batch graph."""
        return [n for n, _ in self.group_plan()]

    GROUP_FORMS = ("columns", "tiled", "persistent")

    def group_plan(self) -> List[Tuple[int, str]]:
        """(items, form) per group of the last built batch graph; form is "columns"
        (per-column launches), "tiled" (tiled column launches) or "persistent" (the
        persistent small-grid sweep kernel)."""
        n = c_int()
        cap = max(1, len(self.problems))
        sizes, form = (c_int * cap)(), (c_int * cap)()
        check(self.lib.nkreg_batch_groups(self._h, byref(n), sizes, form, cap), "nkreg_batch_groups")
        return [(sizes[i], self.GROUP_FORMS[form[i]]) for i in range(n.value)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            for p in getattr(self, "problems", []):
                if not getattr(p, "_owned", True):
                    p._h = None       # the batch destroys the items it owns
            self.lib.nkreg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
