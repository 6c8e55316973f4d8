"""Pins of the oracle's Jacobi-preconditioned CG (NekBone's preconditioner
option, which the paper's benchmark leaves out): the assembled diagonal against
the diagonal of the independently built dense matrix and against the Kronecker
closed form of an affine box; the preconditioned iteration against a dense
solve, with M = I against the unpreconditioned oracle CG step for step, and
with M = diag(A) against textbook CG on the symmetrically scaled system
iterate by iterate."""
import numpy as np
import pytest

import inputs
from oracle import MASS_GWJ, MASS_INVDEG, Mesh, brute


@pytest.mark.parametrize("n,N", [(1, 3), (2, 2), (2, 3), (2, 4)])
@pytest.mark.parametrize("mass", [MASS_GWJ, MASS_INVDEG])
@pytest.mark.parametrize("dirichlet", [False, True])
def test_diagonal_matches_the_dense_matrix(n, N, mass, dirichlet):
    if dirichlet and n * N < 2:
        pytest.skip("no interior node")
    m = Mesh(n, n, n, N, jitter=0.05 if n > 1 else 0.0, seed=13, mass=mass, dirichlet=dirichlet)
    A = brute.dense_matrix(n, n, n, N, m.V, 0.6, mass)
    if dirichlet:
        gx = n * N + 1
        I, J, K = np.meshgrid(np.arange(1, gx - 1), np.arange(1, gx - 1), np.arange(1, gx - 1), indexing="ij")
        keep = (I + gx * (J + gx * K)).ravel(order="F")
        A = A[np.ix_(keep, keep)]
    d = m.diag(0.6)
    assert np.abs(d - np.diag(A)).max() <= 1e-13 * np.abs(np.diag(A)).max()


@pytest.mark.parametrize("nx,ny,nz,N", [(3, 2, 2, 4), (2, 2, 2, 9), (4, 3, 2, 7)])
def test_diagonal_affine_box_closed_form(nx, ny, nz, N):
    """diag(K(x)M(x)M + M(x)K(x)M + M(x)M(x)K + lambda M(x)M(x)M) from the assembled 1D matrices."""
    m = Mesh(nx, ny, nz, N)
    Kx, Mx = brute.assembled_1d(nx, N)
    Ky, My = brute.assembled_1d(ny, N)
    Kz, Mz = brute.assembled_1d(nz, N)
    kx, ky, kz = np.diag(Kx), np.diag(Ky), np.diag(Kz)
    lam = 1.7
    d = (np.einsum("k,j,i->kji", Mz, My, kx) + np.einsum("k,j,i->kji", Mz, ky, Mx) +
         np.einsum("k,j,i->kji", kz, My, Mx) + lam * np.einsum("k,j,i->kji", Mz, My, Mx)).ravel()
    assert np.abs(m.diag(lam) - d).max() <= 1e-13 * np.abs(d).max()


def test_pcg_reaches_the_dense_solution():
    m = Mesh(2, 2, 2, 3, jitter=0.05, seed=3)
    A = brute.dense_matrix(2, 2, 2, 3, m.V, 1.0)
    b = inputs.random_vector(m.NG, 1)
    out = m.pcg(b, 1.0, rtol=1e-14, max_iter=2000)
    assert out["status"] == 0
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(out["x"] - xs) <= 1e-11 * np.linalg.norm(xs)


def test_pcg_with_identity_is_cg():
    m = Mesh(3, 2, 2, 4, jitter=0.05, seed=6)
    b = inputs.random_vector(m.NG, 2)
    p = m.pcg(b, 1.0, fixed_iters=40, inv=np.ones(m.NG))
    c = m.cg(b, 1.0, fixed_iters=40)
    assert p["iters"] == c["iters"] == 40
    assert np.array_equal(p["res"], c["res"]) and np.array_equal(p["x"], c["x"])


def test_jacobi_reduces_iterations_on_a_jittered_box():
    m = Mesh(4, 4, 4, 5, jitter=0.05, seed=9)
    b = inputs.random_vector(m.NG, 3)
    p = m.pcg(b, 1.0, rtol=1e-8, max_iter=5000)
    c = m.cg(b, 1.0, rtol=1e-8, max_iter=5000)
    assert p["status"] == c["status"] == 0
    assert p["iters"] < c["iters"]


@pytest.mark.parametrize("dirichlet", [False, True])
def test_pcg_is_cg_on_the_symmetrically_scaled_system(dirichlet):
    """PCG with M = diag(A) = D is plain CG on D^-1/2 A D^-1/2 y = D^-1/2 b with
    x = D^-1/2 y, and r = D^1/2 r_hat: each of the first 12 iterates and residual
    norms of the oracle's PCG against a textbook dense CG on the scaled system
    (the dense matrix built by the independent brute-force route)."""
    n, N, lam = 2, 4, 0.8
    m = Mesh(n, n, n, N, jitter=0.1, seed=17, dirichlet=dirichlet)
    A = brute.dense_matrix(n, n, n, N, m.V, lam)
    if dirichlet:
        gx = n * N + 1
        I, J, K = np.meshgrid(np.arange(1, gx - 1), np.arange(1, gx - 1), np.arange(1, gx - 1), indexing="ij")
        keep = (I + gx * (J + gx * K)).ravel(order="F")
        A = A[np.ix_(keep, keep)]
    b = inputs.random_vector(m.NG, 21)
    s = 1.0 / np.sqrt(np.diag(A))
    Ah = s[:, None] * A * s[None, :]
    bh = s * b
    y, r = np.zeros_like(bh), bh.copy()
    p, rr = r.copy(), r @ r
    for k in range(1, 13):
        Ap = Ah @ p
        alpha = rr / (p @ Ap)
        y = y + alpha * p
        r = r - alpha * Ap
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        out = m.pcg(b, lam, fixed_iters=k)
        x = s * y
        assert np.linalg.norm(out["x"] - x) <= 1e-10 * np.linalg.norm(x), k
        assert out["res"][k] == pytest.approx(np.linalg.norm(r / s), rel=1e-9), k
