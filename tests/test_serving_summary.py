"""Latency summary of the serving request loops (host arithmetic only)."""
import pytest

from paper_2202_12477_amd import serving


def test_summary_percentiles_and_rate():
    s = serving._summary([1.0, 2.0, 3.0, 4.0], 2.0, 40, {"engine_steps": 7})
    assert s["requests"] == 4 and s["wall_s"] == 2.0 and s["solves_per_s"] == 2.0
    assert s["p50_s"] == pytest.approx(2.5) and s["p99_s"] == pytest.approx(3.97)
    assert s["mean_s"] == pytest.approx(2.5) and s["cg_iterations"] == 40 and s["engine_steps"] == 7
