"""Solver checkpoints: what a beta continuation needs to resume after an interruption.

A continuation measures every level's relative gradient rule against the first level's
||g_0||_inf, so resuming at level i needs the velocity reached after level i - 1, the
beta levels, i and that gradient scale. They are written with ``torch.save`` (tensors and
plain numbers only) and read back with ``weights_only=True`` loading, which executes nothing
from the file. Resuming runs exactly the remaining levels of the uninterrupted solve.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch


def save_continuation(path: str, v: torch.Tensor, betas: Sequence[float], next_level: int, gref_inf: float,
                      reports: Sequence = ()) -> None:
    """Writes the state after levels 0 .. next_level - 1 of a continuation over ``betas``.
    ``gref_inf`` is the first level's ||g_0||_inf (its report's ``gnorm0_inf``)."""
    if not 0 <= next_level <= len(betas):
        raise ValueError("next_level must lie in [0, len(betas)]")
    torch.save({"v": v.detach().to("cpu", torch.float64).clone(), "betas": [float(b) for b in betas],
                "next_level": int(next_level), "gref_inf": float(gref_inf),
                "iterations": [int(r.iterations) for r in reports],
                "cg_iterations": [int(r.cg_iterations) for r in reports]}, path)


def load_continuation(path: str, device: Optional[torch.device] = None) -> dict:
    """Reads a checkpoint written by ``save_continuation``; ``v`` is moved to ``device``."""
    d = torch.load(path, weights_only=True, map_location="cpu")
    for key in ("v", "betas", "next_level", "gref_inf"):
        if key not in d:
            raise ValueError(f"not a continuation checkpoint (no {key!r})")
    if device is not None:
        d["v"] = d["v"].to(device)
    return d


def resume_continuation(problem, path: str, **kw):
    """Runs the levels a checkpoint has not done on ``problem`` (same configuration as the
    interrupted solve); returns (v, reports of those levels)."""
    d = load_continuation(path, problem.device)
    return problem.continuation(d["betas"][d["next_level"]:], v=d["v"], gref_inf=d["gref_inf"], **kw)
