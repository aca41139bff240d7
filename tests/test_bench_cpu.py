"""Host-side checks of bench.py: the one-GPU contract and the counter gate of the roofline."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counters_current():
    text = open(bench.COUNTERS).read()
    block = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    return block["source_sha256"] == bench.source_digest()


def test_counter_summary_covers_both_roofline_kernels_at_the_current_sources():
    """The committed HBM counters cover the column pass that the roofline reports for each
    workload (when they were taken on the kernel sources in the tree; otherwise bench.py
    reports null traffic, which the gate test covers)."""
    if not _counters_current():
        pytest.skip("counters were taken on other kernel sources; bench.py reports traffic as null")
    for sym in ("k_col_w<float, 512, 8, 2>", "k_col_t<float, 256, 16, 2>"):
        t = bench.measured_traffic(sym)
        assert t is not None and t > 0, sym


def test_counter_gate_rejects_other_sources(tmp_path, monkeypatch):
    text = open(bench.COUNTERS).read()
    block = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    block["source_sha256"] = "0" * 64
    stale = tmp_path / "counters.md"
    stale.write_text("# stale\n\n```json\n" + json.dumps(block) + "\n```\n")
    monkeypatch.setattr(bench, "COUNTERS", str(stale))
    assert bench.measured_traffic("k_col_w<float, 512, 8, 2>") is None


def test_counter_traffic_matches_the_algorithmic_bytes():
    """No wasted re-reads. The adjoint stage 1 with the body force reads the divergence
    spectrum, lambda, grad m^j and grad m*_j (2d fields), v (nc d) and F (nc d), and writes
    the accumulator, d spectra and F (nc d): 3 + 3d + 3 nc d fields, i.e. 21 in 3D and 15 in
    2D at nc = 1. Its measured HBM bytes per launch lie within 2% of that."""
    if not _counters_current():
        pytest.skip("counters were taken on other kernel sources")
    for sym, fields, field_bytes in (("k_row_w<float, 256, 4, 5, 3, true>", 21, 256 ** 3 * 4),
                                     ("k_row_w<float, 512, 4, 5, 2, true>", 15, 512 ** 2 * 4)):
        t = bench.measured_traffic(sym)
        alg = fields * field_bytes
        assert abs(t - alg) <= 0.02 * alg, (sym, t, alg)
