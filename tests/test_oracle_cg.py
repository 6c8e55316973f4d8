"""Pins of the oracle's conjugate gradient (Algorithm 1 of arXiv:2202.12477).

Fixed by: a dense solve (numpy.linalg.solve) on tiny systems; CG's defining
properties (monotone A-norm error, Ritz values of the Lanczos tridiagonal
inside A's spectrum, recursive residual equal to b - A x); a manufactured
solution whose discrete error falls spectrally with N; and the feasibility of
the residual-history tolerance used by the GPU parity tests.
"""
import math

import numpy as np
import pytest

import inputs
from oracle import Mesh, brute, rhs


def dense(m, lam):
    I = np.eye(m.NG)
    return np.stack([m.ax(I[:, j], lam) for j in range(m.NG)], axis=1)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_tiny_cg_matches_dense_solve(N):
    m = Mesh(1, 1, 1, N)
    A = brute.dense_matrix(1, 1, 1, N, m.V, 1.0)
    b = rhs(m.NG, 3)
    out = m.cg(b, 1.0, max_iter=10 * m.NG, rtol=1e-15)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(out["x"] - xs) <= 1e-12 * np.linalg.norm(xs)
    # exact arithmetic would finish in N_G steps; allow a few extra for rounding
    assert out["iters"] <= 3 * m.NG


def test_cg_properties_small():
    m = Mesh(2, 2, 2, 2, jitter=0.05, seed=3)
    A = dense(m, 1.0)
    b = rhs(m.NG, 5)
    xs = np.linalg.solve(A, b)
    errs = []
    for k in range(1, 30):
        out = m.cg(b, 1.0, fixed_iters=k)
        e = out["x"] - xs
        errs.append(math.sqrt(e @ A @ e))
        # recursive residual equals the true one (up to rounding)
        rtrue = np.linalg.norm(b - A @ out["x"])
        assert abs(out["res"][-1] - rtrue) <= 1e-10 * np.linalg.norm(b)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    # Lanczos tridiagonal from alpha/beta: Ritz values inside [lmin, lmax]
    out = m.cg(b, 1.0, fixed_iters=20)
    al, be = out["alpha"], out["beta"]
    k = len(al)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1 / al[j] + (be[j - 1] / al[j - 1] if j else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = math.sqrt(be[j]) / al[j]
    ritz = np.linalg.eigvalsh(T)
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ritz.min() >= ev[0] * (1 - 1e-8) and ritz.max() <= ev[-1] * (1 + 1e-8)
    assert abs(ritz.max() - ev[-1]) < 1e-6 * ev[-1]  # the largest converges first


def test_fixed_iterations_and_history_shape():
    c = inputs.PLAIN_SMALL
    m = Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    b = rhs(m.NG, c.rhs_seed)
    out = m.cg(b, c.lam, fixed_iters=100)
    assert out["status"] == 0 and out["iters"] == 100
    assert len(out["res"]) == 101 and out["res"][0] == pytest.approx(np.linalg.norm(b), rel=1e-14)
    assert np.all(out["pap"] > 0)
    # unpreconditioned CG: after 100 iterations the residual has dropped by > 1e3 here
    assert out["res"][-1] < 1e-3 * out["res"][0]


def test_residual_history_envelope():
    """The GPU parity bar for residual histories is 1e-10 relative, widened per
    iteration to 10x the spread between two legitimate CPU summation orders
    (compensated vs plain dot products) where CG's own rounding amplification
    makes 1e-10 unreachable.  Pin that envelope: tight early, wider only late."""
    from cg_envelope import history_bar

    c = inputs.PLAIN_SMALL
    m = Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    b = rhs(m.NG, c.rhs_seed)
    ref, bar = history_bar(m, b, c.lam, 100)
    assert len(ref) == len(bar) == 101
    assert np.all(bar >= 1e-10)
    assert np.all(bar[:80] == 1e-10)   # the first 80 iterations meet 1e-10 as stated
    assert bar.max() < 1e-8            # even the last iterations stay far below one digit


def test_manufactured_solution_converges_spectrally():
    """-lap u + lambda u = f on [0,1]^3 with u = cos(pi x)cos(pi y)cos(pi z) (zero normal
    derivative, natural for an unmasked box) and f = (3 pi^2 + lambda) u.  The discrete
    solution of A u_h = M f must approach u at the nodes spectrally in N."""
    lam = 1.0
    errs = []
    for N in (2, 4, 6, 8):
        m = Mesh(2, 2, 2, N)
        n1 = 2 * N + 1
        g = np.arange(m.NG)
        I, J, K = g % n1, (g // n1) % n1, g // (n1 * n1)
        # affine box: node coordinates from the GLL nodes of each element
        t = np.concatenate([(e + (m.xi[:-1] + 1) / 2) / 2 for e in range(2)] + [[1.0]])
        x, y, z = t[I], t[J], t[K]
        u = np.cos(math.pi * x) * np.cos(math.pi * y) * np.cos(math.pi * z)
        Mdiag = np.zeros(m.NG)
        np.add.at(Mdiag, m.map, m.geo_view()[:, 6, :].ravel())
        out = m.cg(Mdiag * (3 * math.pi ** 2 + lam) * u, lam, max_iter=5000, rtol=1e-13)
        assert out["status"] == 0
        errs.append(np.abs(out["x"] - u).max())
    assert errs[0] > 1e-3
    for a, b in zip(errs, errs[1:]):
        assert b < a / 10, errs
    assert errs[-1] < 1e-6, errs


def test_stored_large_history_pinned():
    """The stored oracle history of the 32^3 N=7 benchmark (tests/golden/cg_history_box32_N7.txt,
    written by make_cg_history.py from the oracle) against an independent route: r_0 = b
    (x0 = 0), and the first iterations of textbook CG with the affine box's Kronecker
    closed form of A (brute.affine_box_ax), which shares no code with oracle.c."""
    from conftest import golden_path

    rows = np.array([[float(v) for v in l.split()] for l in open(golden_path("cg_history_box32_N7.txt"))
                     if l.strip() and not l.startswith("#")])
    c = inputs.PLAIN_LARGE
    assert rows.shape == (c.iters + 1, 4) and np.array_equal(rows[:, 0], np.arange(c.iters + 1))
    href, alt, bar = rows[:, 1], rows[:, 2], rows[:, 3]
    assert np.all(bar >= 1e-10) and np.all(np.abs(href - alt) <= bar * np.abs(href) / 10 + 1e-300)
    b = rhs((c.nx * c.N + 1) ** 3, c.rhs_seed)
    assert href[0] == pytest.approx(np.linalg.norm(b), rel=1e-14)
    k = 3
    x, r = np.zeros_like(b), b.copy()
    p, rho = r.copy(), r @ r
    for j in range(1, k + 1):
        Ap = brute.affine_box_ax(c.nx, c.ny, c.nz, c.N, c.lam, p)
        alpha = rho / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rho, rho_old = r @ r, rho
        p = r + (rho / rho_old) * p
        assert math.sqrt(rho) == pytest.approx(href[j], rel=1e-11), j
