"""Latency summary of the serving request loops (host arithmetic only)."""
import pytest

from paper_2202_12477_amd import serving


def test_summary_percentiles_and_rate():
    s = serving._summary([1.0, 2.0, 3.0, 4.0], 2.0, 40, {"engine_steps": 7})
    assert s["requests"] == 4 and s["wall_s"] == 2.0 and s["solves_per_s"] == 2.0
    assert s["p50_s"] == pytest.approx(2.5) and s["p99_s"] == pytest.approx(3.97)
    assert s["mean_s"] == pytest.approx(2.5) and s["cg_iterations"] == 40 and s["engine_steps"] == 7


def test_budget_counts_and_empty_summary():
    trace = [(0.1, None), (0.5, None), (1.5, None), (2.5, None)]
    e = serving._budget_extra(trace, 2.0, 2.3, 1)
    assert e == {"budget_s": 2.0, "offered": 3, "completed": 1, "backlog": 2, "completed_per_s": 0.5}
    s = serving._summary([], 2.0, 0, e)
    assert s["requests"] == 0 and s["p50_s"] is None and s["backlog"] == 2


def test_window_keeps_the_recipe_and_cuts_at_the_duration():
    import inputs

    w = inputs.serving_window(10.0, 3.0)
    assert w and all(t <= 10.0 for t, _ in w)
    assert [t for t, _ in w] == sorted(t for t, _ in w)
    # the same recipe as the trace: E* in [8, 32768], N in {3,5,7,9,11}
    for _, c in w:
        assert 1 <= c.nx * c.ny * c.nz <= 2 * 32768 and c.N in (3, 5, 7, 9, 11)
