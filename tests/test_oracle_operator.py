"""Pins of the oracle's assembled operator A = Z^T (D^T G D + lambda C) Z
(eq. poisson and eq. stiffness of arXiv:2202.12477).

Each check is fixed by something other than the oracle itself: a dense matrix
built by a different route (oracle/brute.py), the Kronecker closed form of an
affine box, and integrals the SEM reproduces exactly (constants, volume,
linear and quadratic polynomials).  A dropped term, a wrong sign, a transposed
D or a mis-indexed geometric factor fails at least one of them.
"""
import numpy as np
import pytest

import inputs
from oracle import MASS_GWJ, MASS_INVDEG, Mesh, brute


def dense_from_oracle(m, lam):
    I = np.eye(m.NG)
    return np.stack([m.ax(I[:, j], lam) for j in range(m.NG)], axis=1)


@pytest.mark.parametrize("n,N", [(1, N) for N in range(1, 7)] + [(2, N) for N in range(1, 5)])
@pytest.mark.parametrize("mass", [MASS_GWJ, MASS_INVDEG])
def test_brute_force_dense(n, N, mass):
    m = Mesh(n, n, n, N, jitter=0.05 if n > 1 else 0.0, seed=11, mass=mass)
    if n == 1:  # a single element has no interior vertex: distort it by hand
        m.V[7] += [0.03, -0.02, 0.04]
        m.V[2] += [-0.05, 0.01, 0.02]
        from oracle import _p, lib
        lib().oracle_geometry(n, n, n, N, _p(m.V), mass, _p(m.geo))
    lam = 0.7
    A = brute.dense_matrix(n, n, n, N, m.V, lam, mass)
    Ao = dense_from_oracle(m, lam)
    assert np.abs(Ao - A).max() <= 1e-13 * np.abs(A).max()


def test_brute_force_nonsquare_box():
    m = Mesh(3, 2, 1, 2, jitter=0.0, seed=0)
    A = brute.dense_matrix(3, 2, 1, 2, m.V, 2.0)
    Ao = dense_from_oracle(m, 2.0)
    assert np.abs(Ao - A).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("nx,ny,nz,N", [(1, 1, 1, 1), (3, 4, 5, 4), (2, 3, 2, 9), (4, 4, 4, 7), (2, 2, 1, 15)])
def test_affine_box_kronecker_closed_form(nx, ny, nz, N):
    m = Mesh(nx, ny, nz, N)
    x = inputs.random_vector(m.NG, 5)
    y = m.ax(x, 1.3)
    yk = brute.affine_box_ax(nx, ny, nz, N, 1.3, x)
    assert np.linalg.norm(y - yk) <= 1e-13 * np.linalg.norm(yk)


def node_coords(m):
    """Physical coordinates of every global node, from the trilinear map."""
    xi = m.xi
    phi = np.stack([(1 - xi) / 2, (1 + xi) / 2])
    X = np.zeros((m.NG, 3))
    n1 = m.N + 1
    for ez in range(m.nz):
        for ey in range(m.ny):
            for ex in range(m.nx):
                e = ex + m.nx * (ey + m.ny * ez)
                Xe = np.zeros((m.Np, 3))
                for dz in range(2):
                    for dy in range(2):
                        for dx in range(2):
                            v = (ex + dx) + (m.nx + 1) * ((ey + dy) + (m.ny + 1) * (ez + dz))
                            Xe += np.outer(np.kron(phi[dz], np.kron(phi[dy], phi[dx])), m.V[v])
                X[m.map[e * m.Np:(e + 1) * m.Np]] = Xe
    return X


@pytest.fixture(scope="module")
def small_jittered():
    c = inputs.PLAIN_SMALL
    return Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)


def test_symmetry(small_jittered):
    m = small_jittered
    x, y = inputs.random_vector(m.NG, 1), inputs.random_vector(m.NG, 2)
    a, b = x @ m.ax(y, 1.0), y @ m.ax(x, 1.0)
    assert abs(a - b) <= 1e-14 * abs(a) * 10


def test_constants_and_volume(small_jittered):
    """S 1 = 0, so A 1 = lambda M 1, and 1^T M 1 = vol([0,1]^3) = 1 (J has degree <= 2 per axis, N >= 2)."""
    m = small_jittered
    one = np.ones(m.NG)
    S1 = m.ax(one, 0.0)
    scale = np.abs(m.ax(np.abs(inputs.random_vector(m.NG, 3)), 0.0)).max()
    assert np.abs(S1).max() <= 1e-13 * scale
    A1 = m.ax(one, 2.5)
    Mdiag = np.zeros(m.NG)
    np.add.at(Mdiag, m.map, m.geo_view()[:, 6, :].ravel())
    np.testing.assert_allclose(A1, 2.5 * Mdiag, rtol=1e-12, atol=1e-13 * scale)
    assert abs(one @ A1 / 2.5 - 1.0) < 1e-13


def test_inverse_degree_mass_gives_identity():
    """With c = 1/multiplicity (Z^T W Z = I) the operator is A = S + lambda I: A 1 = lambda 1."""
    m = Mesh(3, 2, 4, 3, jitter=0.05, seed=4, mass=MASS_INVDEG)
    A1 = m.ax(np.ones(m.NG), 0.6)
    np.testing.assert_allclose(A1, 0.6, rtol=1e-12, atol=1e-12)


def test_linear_and_mass_exactness(small_jittered):
    """On the jittered N=3 box: for linear p, q with u = I(p), v = I(q):
    u^T S v = grad p . grad q (vol = 1) and u^T M v = integral of p q."""
    m = small_jittered
    X = node_coords(m)
    u, v, one = X[:, 0], X[:, 1], np.ones(m.NG)
    lam = 1.0
    assert abs(u @ m.ax(u, lam) - (1 + lam / 3)) < 1e-12
    assert abs(u @ m.ax(v, lam) - lam / 4) < 1e-12
    assert abs(one @ m.ax(u, lam) - lam / 2) < 1e-12
    w = X[:, 2]
    assert abs(w @ m.ax(w, 0.0) - 1.0) < 1e-12
    assert abs(v @ m.ax(w, 0.0)) < 1e-12


@pytest.mark.parametrize("N", [3, 5])
def test_quadratic_exactness_affine(N):
    """Affine unit box: int |grad x^2|^2 = 4/3, int |grad xy|^2 = 2/3,
    int grad x . grad x^2 = 1, int x^4 = 1/5 (exact for N >= 3)."""
    m = Mesh(3, 2, 2, N)
    X = node_coords(m)
    x, y = X[:, 0], X[:, 1]
    S = lambda a, b: a @ m.ax(b, 0.0)
    assert abs(S(x * x, x * x) - 4 / 3) < 1e-12
    assert abs(S(x * y, x * y) - 2 / 3) < 1e-12
    assert abs(S(x, x * x) - 1.0) < 1e-12
    Mxx = (x * x) @ (m.ax(x * x, 1.0) - m.ax(x * x, 0.0))
    assert abs(Mxx - 1 / 5) < 1e-12


def test_positive_definite_tiny():
    m = Mesh(2, 2, 2, 2, jitter=0.05, seed=9)
    A = dense_from_oracle(m, 1.0)
    np.linalg.cholesky(0.5 * (A + A.T))
    S = dense_from_oracle(m, 0.0)
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert abs(ev[0]) < 1e-12 * ev[-1] and ev[1] > 1e-6 * ev[-1]  # zero eigenvalue is simple (constants)
