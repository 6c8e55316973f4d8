"""Pins of the oracle's Dirichlet box (homogeneous Dirichlet conditions on the
boundary of [0,1]^3, the setting of the paper's experiments, whose DOF counts
are (nN-1)^3): the boundary nodes carry no DOF, so the operator is the
restriction R A R^T of the unmasked operator to the interior nodes.

Pinned by the restriction of the independently built dense matrix
(oracle/brute.py), by the Kronecker closed form of an affine box with the 1D
matrices restricted to interior nodes, by the loss of the constant null space
(the masked stiffness is positive definite), and by spectral convergence to a
manufactured solution that vanishes on the boundary.
"""
import math

import numpy as np
import pytest

import inputs
from oracle import MASS_GWJ, MASS_INVDEG, Mesh, brute


def interior(nx, ny, nz, N):
    """Lexicographic global indices (unmasked numbering) of the interior nodes."""
    gx, gy, gz = nx * N + 1, ny * N + 1, nz * N + 1
    I, J, K = np.meshgrid(np.arange(1, gx - 1), np.arange(1, gy - 1), np.arange(1, gz - 1), indexing="ij")
    return (I + gx * (J + gy * K)).ravel(order="F")


def dense(m, lam):
    I = np.eye(m.NG)
    return np.stack([m.ax(I[:, j], lam) for j in range(m.NG)], axis=1)


@pytest.mark.parametrize("n,N", [(2, 1), (2, 2), (2, 3), (3, 2), (2, 4)])
@pytest.mark.parametrize("mass", [MASS_GWJ, MASS_INVDEG])
def test_dirichlet_is_the_restricted_dense_matrix(n, N, mass):
    m = Mesh(n, n, n, N, jitter=0.05, seed=21, mass=mass, dirichlet=True)
    assert m.NG == (n * N - 1) ** 3
    keep = interior(n, n, n, N)
    A = brute.dense_matrix(n, n, n, N, m.V, 0.8, mass)[np.ix_(keep, keep)]
    Ao = dense(m, 0.8)
    assert np.abs(Ao - A).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("nx,ny,nz,N", [(2, 2, 2, 2), (3, 4, 2, 4), (2, 3, 2, 9), (4, 4, 4, 7), (2, 2, 1, 15)])
def test_dirichlet_affine_box_kronecker_closed_form(nx, ny, nz, N):
    m = Mesh(nx, ny, nz, N, dirichlet=True)
    keep = interior(nx, ny, nz, N)
    x = inputs.random_vector(m.NG, 7)
    xf = np.zeros((nx * N + 1) * (ny * N + 1) * (nz * N + 1))
    xf[keep] = x
    yk = brute.affine_box_ax(nx, ny, nz, N, 1.1, xf)[keep]
    y = m.ax(x, 1.1)
    assert np.linalg.norm(y - yk) <= 1e-13 * np.linalg.norm(yk)


def test_dirichlet_stiffness_is_positive_definite():
    """Without boundary masking S.1 = 0; with it the constants are not in the
    space and S_D is positive definite (smallest eigenvalue bounded away from 0,
    about 3 pi^2 times the smallest mass entry scale)."""
    m = Mesh(2, 2, 2, 3, jitter=0.05, seed=4, dirichlet=True)
    S = dense(m, 0.0)
    assert np.abs(S - S.T).max() <= 1e-13 * np.abs(S).max()
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev[0] > 1e-2 * ev[-1] / m.NG


def test_dirichlet_manufactured_solution_converges_spectrally():
    """u = sin(pi x) sin(pi y) sin(pi z) vanishes on the boundary; A u_h = M f with
    f = (3 pi^2 + lambda) u.  The nodal error must fall by orders of magnitude as
    N grows on a fixed 2^3 jittered mesh."""
    lam, errs = 1.0, []
    for N in (2, 4, 6, 8):
        m = Mesh(2, 2, 2, N, jitter=0.05, seed=8, dirichlet=True)
        full = Mesh(2, 2, 2, N, jitter=0.05, seed=8)
        X = node_coords(full)[interior(2, 2, 2, N)]
        u = np.sin(math.pi * X[:, 0]) * np.sin(math.pi * X[:, 1]) * np.sin(math.pi * X[:, 2])
        # M f: the mass term alone (the lumped GLL mass, diagonal), from the operator with S removed
        Mdiag = m.ax(np.ones(m.NG), 1.0) - m.ax(np.ones(m.NG), 0.0)
        b = Mdiag * (3 * math.pi ** 2 + lam) * u
        out = m.cg(b, lam, max_iter=5000, rtol=1e-13)
        assert out["status"] == 0
        errs.append(np.abs(out["x"] - u).max())
    assert errs[0] > 10 * errs[1] > 100 * errs[2] and errs[3] < 1e-6, errs


def node_coords(m):
    """Physical coordinates of every global node of an unmasked mesh, from the trilinear map."""
    xi = m.xi
    phi = np.stack([(1 - xi) / 2, (1 + xi) / 2])
    X = np.zeros((m.NG, 3))
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


def test_dirichlet_dof_counts_match_the_paper_formula():
    """(nN-1)^3 DOFs, the paper's counts (tests/test_metrics.py pins them against its tables)."""
    for nx, ny, nz, N in ((4, 4, 4, 3), (2, 3, 4, 5), (1, 2, 2, 7)):
        m = Mesh(nx, ny, nz, N, dirichlet=True)
        assert m.NG == (nx * N - 1) * (ny * N - 1) * (nz * N - 1)
        assert int((m.map >= 0).sum()) == m.NL - int((m.map < 0).sum())
        assert set(np.unique(m.map[m.map >= 0])) == set(range(m.NG))
