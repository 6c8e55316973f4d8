"""The oracle's timing build (the benchmark's CPU baseline) computes what the
parity build computes.

The timing build sweeps the elements in 8 classes of a box, (ex mod 2, ey mod 2,
ez mod 2), on several threads: that is race-free only if no two elements of a
class share a global node, which is checked here on the map.  Its operator and
its CG residual history must then agree with the single-threaded parity build
up to summation order (operator 1e-14; history within the envelope used for
the GPU).
"""
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from cg_envelope import compare_history, history_bar


def openmp_available():
    if not shutil.which("gcc"):
        return False
    r = subprocess.run(["gcc", "-fopenmp", "-x", "c", "-", "-o", "/dev/null"], input="int main(){return 0;}",
                       capture_output=True, text=True)
    return r.returncode == 0


pytestmark = pytest.mark.skipif(not openmp_available(), reason="gcc with OpenMP not available")


@pytest.fixture(scope="module")
def tlib():
    L = oracle.timing_lib(build=True)
    L.oracle_set_threads(4)
    yield L
    L.oracle_set_threads(1)


@pytest.mark.parametrize("dims,N,dirichlet", [((3, 4, 5), 2, False), ((4, 3, 2), 3, True), ((5, 1, 2), 4, False)])
def test_classes_share_no_node(dims, N, dirichlet):
    m = oracle.Mesh(*dims, N, jitter=0.05, seed=3, dirichlet=dirichlet)
    order, off = m.classes()
    assert sorted(order.tolist()) == list(range(m.E)) and off[0] == 0 and off[-1] == m.E
    mp = m.map.reshape(m.E, m.Np)
    for k in range(8):
        els = order[off[k]:off[k + 1]]
        nodes = mp[els].ravel()
        nodes = nodes[nodes >= 0]
        assert len(np.unique(nodes)) == len(nodes), f"class {k} shares a node"


@pytest.mark.parametrize("N,jitter", [(1, 0.05), (3, 0.05), (7, 0.0)])
def test_timing_operator_equals_parity_operator(tlib, N, jitter):
    m = oracle.Mesh(5, 4, 6, N, jitter=jitter, seed=9)
    x = np.random.default_rng(N).standard_normal(m.NG)
    y = m.ax(x, 1.0)
    assert np.linalg.norm(m.ax_classes(x, 1.0, L=tlib) - y) <= 1e-14 * np.linalg.norm(y)


def test_timing_cg_history_within_envelope(tlib):
    m = oracle.Mesh(4, 4, 4, 3, jitter=0.05, seed=1)
    b = oracle.rhs(m.NG, 2)
    href, bar = history_bar(m, b, 1.0, 100)
    got = m.cg_classes(b, 1.0, fixed_iters=100, L=tlib)["res"]
    assert compare_history(got, href, bar) <= 1.0
