"""Pins of the oracle's 1D building blocks: GLL nodes/weights, derivative matrix,
1D stiffness, and the counter-based random generator.

Closed forms are textbook (Canuto et al.; Deville, Fischer & Mund, cited by the
paper for the SEM operators); the random-generator values are splitmix64's
published test vectors (tests/golden/splitmix64_vectors.txt).
"""
import math

import numpy as np
import pytest

from conftest import golden_path
from oracle import brute

S5 = 1 / math.sqrt(5.0)
S37 = math.sqrt(3.0 / 7.0)
GLL_CLOSED = {
    1: ([-1, 1], [1, 1]),
    2: ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1, -S5, S5, 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1, -S37, 0, S37, 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_forms(oracle_mod, N):
    xi, w = oracle_mod.gll(N)
    xe, we = GLL_CLOSED[N]
    np.testing.assert_allclose(xi, xe, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, we, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 16))
def test_gll_quadrature_exactness(oracle_mod, N):
    """GLL with N+1 points integrates x^k exactly on [-1,1] for k <= 2N-1."""
    xi, w = oracle_mod.gll(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(0, 2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 2e-14, (N, k)
    # not exact at degree 2N (the GLL rule's known deficiency)
    k = 2 * N
    assert abs(np.dot(w, xi ** k) - 2.0 / (k + 1)) > 1e-10


@pytest.mark.parametrize("N", range(1, 16))
def test_gll_matches_companion_matrix_route(oracle_mod, N):
    xi, w = oracle_mod.gll(N)
    xb, wb = brute.gll(N)
    np.testing.assert_allclose(xi, xb, rtol=0, atol=1e-13)
    np.testing.assert_allclose(w, wb, rtol=1e-12, atol=0)


def test_deriv_closed_forms(oracle_mod):
    np.testing.assert_allclose(oracle_mod.deriv(1), [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-15)
    np.testing.assert_allclose(oracle_mod.deriv(2), [[-1.5, 2, -0.5], [-0.5, 0, 0.5], [0.5, -2, 1.5]], atol=1e-15)


@pytest.mark.parametrize("N", range(1, 16))
def test_deriv_differentiates_polynomials(oracle_mod, N):
    """D xi^k = k xi^(k-1) exactly for k <= N; D 1 = 0; corners are -+N(N+1)/4."""
    xi, _ = oracle_mod.gll(N)
    D = oracle_mod.deriv(N)
    scale = np.abs(D).max()
    assert np.abs(D @ np.ones(N + 1)).max() < 1e-13 * scale
    for k in range(1, N + 1):
        np.testing.assert_allclose(D @ xi ** k, k * xi ** (k - 1), atol=1e-12 * scale * k)
    assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-14 * N * N
    assert abs(D[N, N] - N * (N + 1) / 4) < 1e-14 * N * N
    np.testing.assert_allclose(D, brute.deriv(N, xi), atol=1e-11 * scale)


def test_1d_stiffness_closed_forms(oracle_mod):
    """K = D^T W D equals the exact integral of l_i' l_j' (degree 2N-2 <= 2N-1)."""
    for N, K in [(1, 0.5 * np.array([[1, -1], [-1, 1]])),
                 (2, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 6.0)]:
        _, w = oracle_mod.gll(N)
        D = oracle_mod.deriv(N)
        np.testing.assert_allclose(D.T @ np.diag(w) @ D, K, atol=1e-14)


def test_splitmix64_published_vectors(oracle_mod):
    rows = [l.split() for l in open(golden_path("splitmix64_vectors.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 8
    for s, i, v in rows:
        assert oracle_mod.splitmix64(int(s), int(i)) == int(v)


def test_uniform_and_rhs(oracle_mod):
    b = oracle_mod.rhs(100000, 7)
    assert b.min() >= -1.0 and b.max() < 1.0
    assert abs(b.mean()) < 0.01 and abs(b.var() - 1 / 3) < 0.01
    assert np.array_equal(b, oracle_mod.rhs(100000, 7))
    assert not np.array_equal(b, oracle_mod.rhs(100000, 8))
    # a value is a function of (seed, stream, index) only
    u = oracle_mod.uniform(7, 0, 12345)
    assert b[12345] == 2.0 * u - 1.0
    # the stream's start state is output number `stream` of the seed's sequence
    start = oracle_mod.splitmix64(7, 0)
    assert u == (oracle_mod.splitmix64(start, 12345) >> 11) * 2.0 ** -53


def test_vertices_jitter(oracle_mod):
    nx, ny, nz = 4, 3, 5
    V0 = oracle_mod.vertices(nx, ny, nz, 0.0, 1)
    V = oracle_mod.vertices(nx, ny, nz, 0.05, 1)
    idx = np.arange(V.shape[0])
    i, j, k = idx % (nx + 1), (idx // (nx + 1)) % (ny + 1), idx // ((nx + 1) * (ny + 1))
    np.testing.assert_array_equal(V0, np.stack([i / nx, j / ny, k / nz], 1))
    interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
    np.testing.assert_array_equal(V[~interior], V0[~interior])
    h = np.array([1 / nx, 1 / ny, 1 / nz])
    d = (V - V0)[interior] / h
    assert np.all(np.abs(d) <= 0.05) and np.all(np.abs(d) > 0)
    assert np.array_equal(V, oracle_mod.vertices(nx, ny, nz, 0.05, 1))
