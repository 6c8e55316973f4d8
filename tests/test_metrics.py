"""The reporting formulas reproduce the paper's printed data (arXiv:2202.12477).

- FOM (eq. nekbone_flops) recomputed from the printed single-rank throughput
  (eq. throughput) matches the printed FOM of the same run to the 3-digit
  rounding of the throughput (Fig. CrusherScalingP7/P15 vs CrusherThroughputP7/P15);
  the printed DOF counts are (nN-1)^3, i.e. the runs mask a Dirichlet boundary.
- eq. (op_perf) equals the roofline expression plotted in Fig. MI250XOperator,
  and every measured operator point sits under it.
"""
import numpy as np
import pytest

from conftest import golden_path
from paper_2202_12477_amd import metrics


def _rows(name):
    return [list(map(float, l.split())) for l in open(golden_path(name)) if l.strip() and not l.startswith("#")]


def test_fom_from_throughput_matches_printed_fom():
    rows = _rows("crusher_single_rank.txt")
    assert len(rows) == 22
    for N, dofs, fom_printed, thr in rows:
        N, dofs = int(N), int(dofs)
        n = metrics.masked_box_elements(dofs, N)
        E = n ** 3
        seconds = dofs * 100 / thr  # one rank
        assert metrics.throughput(dofs, 100, 1, seconds) == pytest.approx(thr, rel=1e-12)
        fom = metrics.fom(E, N, 100, seconds) / 1e9
        assert fom == pytest.approx(fom_printed, rel=6e-3), (N, dofs)


def test_op_roofline_matches_plotted_expression():
    rows = _rows("operator_roofline_mi250x.txt")
    for N, measured in rows:
        x = N
        plotted = 1117 * ((12 * (x + 1) + 18) * (x + 1) ** 3) / ((68 * (x + 1) ** 3 + 8 * (x) ** 3))
        assert metrics.op_roofline(int(N), 1117.0) == pytest.approx(plotted, rel=1e-14)
        assert measured <= plotted
    assert metrics.op_roofline(7, 1117.0) == pytest.approx(1735.8, abs=0.05)
    assert metrics.op_roofline(7, 1117.0, C=100.0) == 100.0


def test_byte_models():
    # paper's CG bytes are the operator (8NG+68NL), gather (12NG+12NL) and 11 vector passes (88NG)
    NG, NL = 11390625, 16777216
    assert metrics.cg_iter_bytes_paper(NG, NL) == metrics.ax_bytes_paper(NG, NL) + 12 * NG + 12 * NL + 88 * NG
    assert metrics.ax_bytes_fused(NG, NL) == pytest.approx(1.189e9, rel=1e-3)
    assert metrics.ax_flops(32768, 7) == pytest.approx(1.91e9, rel=1e-2)
    # NekBone and hipBone FLOP counts share the leading term
    assert metrics.nekbone_flops(1, 15) - metrics.hipbone_cg_flops(1, 15) == 34 * 16 ** 3 - 19 * 16 ** 3 - 10 * 15 ** 3
