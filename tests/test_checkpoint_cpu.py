"""Continuation checkpoints on the CPU: round trip through torch.save / weights_only loading,
argument checks, and refusal of files that are not checkpoints."""
import pytest
import torch

from paper_1408_6299_amd import checkpoint as ck


class _Rep:
    iterations, cg_iterations = 5, 24


def test_round_trip(tmp_path):
    v = torch.randn(2, 16, 16, dtype=torch.float64)
    p = str(tmp_path / "c.pt")
    ck.save_continuation(p, v, [1e-1, 1e-2, 1e-3], 2, 0.125, [_Rep(), _Rep()])
    d = ck.load_continuation(p)
    assert torch.equal(d["v"], v) and d["v"].dtype == torch.float64
    assert d["betas"] == [1e-1, 1e-2, 1e-3] and d["next_level"] == 2 and d["gref_inf"] == 0.125
    assert d["iterations"] == [5, 5] and d["cg_iterations"] == [24, 24]


def test_bad_level_and_foreign_file(tmp_path):
    with pytest.raises(ValueError):
        ck.save_continuation(str(tmp_path / "x.pt"), torch.zeros(2, 4, 4), [1.0], 3, 1.0)
    p = str(tmp_path / "y.pt")
    torch.save({"something": torch.zeros(3)}, p)
    with pytest.raises(ValueError):
        ck.load_continuation(p)
