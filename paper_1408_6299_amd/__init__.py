"""MI355X (gfx950) Gauss-Newton-Krylov diffeomorphic registration (Mang & Biros, arXiv 1408.6299).

The computation lives in the HIP library ``libnkreg.so`` (C ABI in
``include/nkreg.h``); this package only marshals torch tensors into it.
Importing the package loads the library and raises if it has not been built.
"""
from ._lib import NkregError, load as _load

_load()

from .api import Batch, BetaSearchResult, BetaTrial, Problem, SolveResult, launch_floor  # noqa: E402
from .autograd import RegistrationObjective, objective  # noqa: E402
from .checkpoint import load_continuation, resume_continuation, save_continuation  # noqa: E402

__all__ = ["Problem", "Batch", "SolveResult", "BetaSearchResult", "BetaTrial", "NkregError", "RegistrationObjective",
           "objective", "save_continuation", "load_continuation", "resume_continuation", "launch_floor"]
