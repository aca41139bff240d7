"""ctypes declarations of the C ABI in include/nkreg.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_int, c_longlong, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnkreg.so")

OK, EINVAL, ESHAPE, ENOMEM, EHIP, ESTATE, ENONFINITE, ECFL, ENOCONV, ENOTIMPL = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)


class Config(Structure):
    _fields_ = [("dim", c_int), ("n", c_int * 3), ("nt", c_int), ("nc", c_int), ("reg", c_int),
                ("incompressible", c_int), ("beta", c_double), ("precision", c_int),
                ("checkpoint_every", c_int), ("cfl_max", c_double),
                ("trajectory_slots", c_int)]


HISTORY_COLS = 11    # NKREG_HISTORY_COLS


class SolveOpts(Structure):
    _fields_ = [("max_outer", c_int), ("gtol", c_double), ("tau_J", c_double), ("pcg_maxit", c_int),
                ("cfl_guard", c_int), ("verbose", c_int), ("gref_inf", c_double),
                ("h_history", POINTER(c_double)), ("history_cap", c_int), ("history_detf", c_int)]


class SolveReport(Structure):
    _fields_ = [("iterations", c_int), ("cg_iterations", c_int), ("n_pde", c_int),
                ("line_search_failed", c_int), ("converged", c_int), ("J0", c_double), ("J", c_double),
                ("J_dist", c_double), ("J_reg", c_double), ("gnorm0_inf", c_double),
                ("gnorm_inf", c_double), ("seconds", c_double), ("stop_reason", c_int), ("history_rows", c_int)]


class PicardOpts(Structure):
    _fields_ = [("memory", c_int), ("stagnation_count", c_int), ("stagnation_tol", c_double)]


MAX_BETA_TRIALS = 64


class BetaSearchOpts(Structure):
    _fields_ = [("eps_F", c_double), ("beta_start", c_double), ("beta_min", c_double), ("dbeta_rel", c_double),
                ("l2_rel_min", c_double), ("max_steps", c_int), ("solve", SolveOpts)]


class BetaSearchReport(Structure):
    _fields_ = [("steps", c_int), ("breached", c_int), ("reason", c_int), ("beta_star", c_double),
                ("min_det_star", c_double), ("l2_rel_star", c_double), ("dbeta_min", c_double),
                ("newton_iterations", c_int), ("cg_iterations", c_int), ("seconds", c_double),
                ("trial_beta", c_double * MAX_BETA_TRIALS), ("trial_min_det", c_double * MAX_BETA_TRIALS),
                ("trial_l2_rel", c_double * MAX_BETA_TRIALS), ("trial_accepted", c_int * MAX_BETA_TRIALS)]


# name -> (restype, argtypes); every symbol declared in include/nkreg.h
SIGNATURES = {
    "nkreg_version": (c_char_p, []),
    "nkreg_status_string": (c_char_p, [c_int]),
    "nkreg_last_error": (c_char_p, []),
    "nkreg_create": (c_int, [POINTER(Config), c_void_p, POINTER(c_void_p)]),
    "nkreg_destroy": (c_int, [c_void_p]),
    "nkreg_set_beta": (c_int, [c_void_p, c_double]),
    "nkreg_set_hessian": (c_int, [c_void_p, c_int]),
    "nkreg_hessian_assemble": (c_int, [c_void_p, c_void_p]),
    "nkreg_hessian_lanczos": (c_int, [c_void_p, c_int, POINTER(c_double), POINTER(c_int)]),
    "nkreg_use_graphs": (c_int, [c_void_p, c_int]),
    "nkreg_describe": (c_int, [c_void_p, ctypes.c_char_p, c_int]),
    "nkreg_set_images": (c_int, [c_void_p, c_void_p, c_void_p]),
    "nkreg_forward": (c_int, [c_void_p, c_void_p, c_void_p]),
    "nkreg_objective_gradient": (c_int, [c_void_p, c_void_p, POINTER(c_double), POINTER(c_double),
                                         POINTER(c_double), c_void_p]),
    "nkreg_objective": (c_int, [c_void_p, c_void_p, POINTER(c_double), POINTER(c_double),
                                POINTER(c_double)]),
    "nkreg_hessian_matvec": (c_int, [c_void_p, c_void_p, c_void_p]),
    "nkreg_precond_apply": (c_int, [c_void_p, c_void_p, c_void_p]),
    "nkreg_project": (c_int, [c_void_p, c_void_p, c_void_p]),
    "nkreg_pcg": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, POINTER(c_int),
                          POINTER(c_double)]),
    "nkreg_det_grad_y": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
    "nkreg_newton_solve": (c_int, [c_void_p, c_void_p, POINTER(SolveOpts), POINTER(SolveReport)]),
    "nkreg_picard_solve": (c_int, [c_void_p, c_void_p, POINTER(SolveOpts), POINTER(PicardOpts),
                                   POINTER(SolveReport)]),
    "nkreg_continuation": (c_int, [c_void_p, c_void_p, POINTER(c_double), c_int, POINTER(SolveOpts),
                                   POINTER(SolveReport)]),
    "nkreg_beta_search": (c_int, [c_void_p, c_void_p, POINTER(BetaSearchOpts), POINTER(BetaSearchReport)]),
    "nkreg_gradient": (c_int, [c_void_p, c_void_p, c_void_p]),
    "nkreg_divergence": (c_int, [c_void_p, c_void_p, c_void_p]),
    "nkreg_apply_reg": (c_int, [c_void_p, c_void_p, c_void_p]),
    "nkreg_dot": (c_int, [c_void_p, c_void_p, c_void_p, c_longlong, POINTER(c_double)]),
    "nkreg_timer_arm": (c_int, [c_void_p, c_int, c_int]),
    "nkreg_matvec_bytes": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_double), POINTER(c_int)]),
    "nkreg_timer_read": (c_int, [c_void_p, POINTER(c_int), POINTER(c_double), POINTER(c_double)]),
    "nkreg_exchange_canary": (c_int, [c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_int, c_void_p]),
    "nkreg_launch_floor": (c_int, [c_int, c_int, c_int, c_int, c_void_p, ctypes.POINTER(c_double)]),
    "nkreg_gradient_noalloc": (c_int, [c_int, POINTER(c_int), c_int, c_void_p, c_void_p, c_void_p]),
    "nkreg_batch_create": (c_int, [c_int, POINTER(Config), c_void_p, POINTER(c_void_p)]),
    "nkreg_batch_wrap": (c_int, [c_int, POINTER(c_void_p), POINTER(c_void_p)]),
    "nkreg_batch_item": (c_int, [c_void_p, c_int, POINTER(c_void_p)]),
    "nkreg_batch_objective_gradient": (c_int, [c_void_p, POINTER(c_void_p), POINTER(c_double), POINTER(c_double),
                                               POINTER(c_double), POINTER(c_void_p)]),
    "nkreg_batch_set_state": (c_int, [c_void_p, POINTER(c_void_p)]),
    "nkreg_batch_pcg": (c_int, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), c_double, c_int, POINTER(c_int),
                                POINTER(c_double)]),
    "nkreg_batch_groups": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_int), c_int]),
    "nkreg_batch_destroy": (c_int, [c_void_p]),
    "nkreg_batch_hessian_matvec": (c_int, [c_void_p, POINTER(c_void_p), POINTER(c_void_p)]),
}

_lib = None


class NkregError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libnkreg.so (built by paper_1408_6299_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    # torch's HIP runtime must be loaded first: libnkreg.so then binds to that
    # runtime instead of bringing a second HIP/HSA runtime into the process,
    # which leaves the device invisible to one of them.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python __graft_entry__.py` or `python paper_1408_6299_amd/build.py` "
                          "(the HIP library is required; there is no fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str) -> int:
    if status == OK:
        return status
    lib = load()
    detail = lib.nkreg_last_error().decode() or lib.nkreg_status_string(status).decode()
    raise NkregError(status, where, detail)
