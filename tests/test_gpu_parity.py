"""GPU parity of the HIP path against the oracle, through the C ABI.

Bars: integer data (forcing bits, map) bit-exact; geometric factors and the 1D
basis within 1e-14 relative (two independent FP64 computations of the same
closed forms); y = A x within 1e-12 relative in the 2-norm; CG residual
histories within the per-iteration envelope of tests/cg_envelope.py (1e-10,
widened only where the oracle's own two summation orders drift apart).
"""
import sys

import numpy as np
import pytest

import inputs
import oracle
from cg_envelope import compare_history, history_bar
from conftest import golden_path
from oracle import brute

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2202_12477_amd as hb  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def make(nx, ny, nz, N, jitter=0.05, seed=1, mass=0):
    say(f"[case] mesh {nx}x{ny}x{nz} N={N} jitter={jitter} seed={seed} mass={mass}")
    return hb.Mesh(nx, ny, nz, N, jitter=jitter, seed=seed, mass=mass), oracle.Mesh(nx, ny, nz, N, jitter=jitter,
                                                                                      seed=seed, mass=mass)


@pytest.mark.parametrize("n,seed", [(1, 0), (1000, 3), (2197, 2), (1 << 20, 99)])
def test_rhs_bit_exact(n, seed):
    say(f"[case] rhs n={n} seed={seed}")
    b = torch.empty(n, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, seed)
    assert np.array_equal(host(b), oracle.rhs(n, seed))


@pytest.mark.parametrize("N", [1, 2, 3, 7, 8, 15])
def test_basis_and_geometry(N):
    m, ref = make(3, 2, 2, N, jitter=0.05, seed=7)
    geo, mp, D, xi, w = m.export()
    np.testing.assert_array_equal(mp.ravel(), ref.map)
    np.testing.assert_allclose(xi, ref.xi, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, ref.w, rtol=1e-14)
    np.testing.assert_allclose(D, ref.D, rtol=0, atol=1e-14 * np.abs(ref.D).max())
    g_ref = ref.geo_view()
    for f in range(7):
        scale = np.abs(g_ref[:, f]).max()
        assert np.abs(geo[:, f] - g_ref[:, f]).max() <= 1e-14 * scale * 4, f


def test_inverse_degree_geometry():
    m, ref = make(3, 3, 2, 4, mass=1)
    geo, _, _, _, _ = m.export()
    np.testing.assert_allclose(geo[:, 6], ref.geo_view()[:, 6], rtol=1e-15)


# Small meshes with ragged tails: E is not a multiple of the elements packed per block.
AX_CASES = [(1, 1, 1, 1), (3, 2, 5, 1), (4, 4, 4, 3), (5, 3, 2, 2), (3, 3, 3, 4), (2, 3, 4, 5), (3, 2, 2, 6),
            (3, 3, 2, 7), (2, 2, 3, 8), (2, 1, 2, 9), (1, 2, 2, 10), (2, 1, 1, 11), (1, 1, 2, 12), (1, 2, 1, 13),
            (1, 1, 1, 14), (2, 1, 1, 15), (7, 1, 1, 3)]


@pytest.mark.parametrize("nx,ny,nz,N", AX_CASES)
def test_ax_matches_oracle(nx, ny, nz, N):
    m, ref = make(nx, ny, nz, N, jitter=0.05 if min(nx, ny, nz) > 1 else 0.0, seed=nx + 10 * N)
    x = inputs.random_vector(m.NG, N)
    y = torch.full((m.NG,), float("nan"), dtype=torch.float64, device=DEV)  # y is overwritten, not accumulated
    m.ax(1.3, dev(x), y)
    assert relerr(host(y), ref.ax(x, 1.3)) <= 1e-12


def test_ax_inverse_degree_mass():
    m, ref = make(4, 3, 2, 5, mass=1)
    x = inputs.random_vector(m.NG, 4)
    y = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    m.ax(0.8, dev(x), y)
    assert relerr(host(y), ref.ax(x, 0.8)) <= 1e-12


def test_ax_small_config_and_invariants():
    c = inputs.PLAIN_SMALL
    m, ref = make(c.nx, c.ny, c.nz, c.N, c.jitter, c.mesh_seed)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    y = torch.empty_like(b)
    m.ax(c.lam, b, y)
    assert relerr(host(y), ref.ax(oracle.rhs(m.NG, c.rhs_seed), c.lam)) <= 1e-12
    # symmetry and A 1 = lambda M 1 on the device output
    u, v = dev(inputs.random_vector(m.NG, 1)), dev(inputs.random_vector(m.NG, 2))
    Au, Av = torch.empty_like(u), torch.empty_like(u)
    m.ax(1.0, u, Au)
    m.ax(1.0, v, Av)
    a, bb = float(torch.dot(v, Au)), float(torch.dot(u, Av))
    assert abs(a - bb) <= 1e-13 * abs(a)
    one = torch.ones_like(u)
    A1 = torch.empty_like(u)
    m.ax(1.0, one, A1)
    assert abs(float(A1.sum()) - 1.0) < 1e-13  # 1^T A 1 = lambda * volume


def test_ax_large_config_full():
    """32^3 affine elements at N=7 (11.4M DOFs): the whole output against the oracle
    and against the Kronecker closed form of the affine box."""
    c = inputs.PLAIN_LARGE
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    say("[case] large config Ax")
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    y = torch.empty_like(b)
    m.ax(c.lam, b, y)
    yg = host(y)
    bh = oracle.rhs(m.NG, c.rhs_seed)
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    assert relerr(yg, ref.ax(bh, c.lam)) <= 1e-12
    del ref
    assert relerr(yg, brute.affine_box_ax(c.nx, c.ny, c.nz, c.N, c.lam, bh)) <= 1e-12
    # repeated application is stable to rounding (atomics change only the summation order)
    y2 = torch.empty_like(b)
    m.ax(c.lam, b, y2)
    assert relerr(host(y2), yg) <= 1e-14
    m.close()


def test_cg_small_config_history():
    c = inputs.PLAIN_SMALL
    m, ref = make(c.nx, c.ny, c.nz, c.N, c.jitter, c.mesh_seed)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    x = torch.full_like(b, float("nan"))  # x0_zero ignores the initial content
    res = m.cg(c.lam, b, x, max_iter=c.iters, fixed_iters=True)
    assert res.status == hb.HB_OK and res.iters == c.iters
    bh = oracle.rhs(m.NG, c.rhs_seed)
    href, bar = history_bar(ref, bh, c.lam, c.iters)
    ratio = compare_history(res.history, href, bar)
    say(f"history ratio to bar: {ratio:.3f}")
    assert ratio <= 1.0
    out = ref.cg(bh, c.lam, fixed_iters=c.iters)
    # the iterate itself: same to the accuracy the residual history allows
    assert relerr(host(x), out["x"]) <= 1e-8
    assert res.res0 == pytest.approx(out["res"][0], rel=1e-14)


def test_cg_tolerance_mode_and_restart():
    m, ref = make(3, 3, 3, 4, jitter=0.05, seed=5)
    bh = oracle.rhs(m.NG, 11)
    b = dev(bh)
    x = torch.zeros_like(b)
    res = m.cg(1.0, b, x, max_iter=2000, fixed_iters=False, rtol=1e-8, check_every=10)
    out = ref.cg(bh, 1.0, max_iter=2000, rtol=1e-8)
    assert res.status == hb.HB_OK and out["status"] == 0
    assert abs(res.iters - out["iters"]) <= 1
    assert res.res <= 1e-8 * res.bnorm
    # true residual from the oracle operator
    xr = host(x)
    assert np.linalg.norm(bh - ref.ax(xr, 1.0)) <= 2e-8 * np.linalg.norm(bh)
    # restart from the solution with a non-zero initial guess: converges immediately
    res2 = m.cg(1.0, b, x, max_iter=50, fixed_iters=False, rtol=1e-7, x0_zero=False)
    assert res2.status == hb.HB_OK and res2.iters == 0
    # a cap below the needed count reports NOT_CONVERGED with the history filled
    x.zero_()
    res3 = m.cg(1.0, b, x, max_iter=5, fixed_iters=False, rtol=1e-12)
    assert res3.status == hb.HB_ERR_NOT_CONVERGED and res3.iters == 5 and len(res3.history) == 6


def test_cg_edge_cases():
    m, ref = make(1, 1, 1, 1, jitter=0.0)
    b = dev(oracle.rhs(m.NG, 3))
    x = torch.zeros_like(b)
    # zero iterations
    r0 = m.cg(1.0, b, x, max_iter=0, fixed_iters=True)
    assert r0.status == hb.HB_OK and r0.iters == 0 and len(r0.history) == 1
    # zero right-hand side: r0 = 0 stops at once with x = 0
    z = torch.zeros_like(b)
    rz = m.cg(1.0, z, x, max_iter=10, fixed_iters=True)
    assert rz.status == hb.HB_OK and rz.iters == 0 and float(x.abs().max()) == 0.0
    # non-finite forcing
    bn = b.clone()
    bn[3] = float("nan")
    rn = m.cg(1.0, bn, x, max_iter=10, fixed_iters=True)
    assert rn.status == hb.HB_ERR_NONFINITE and rn.iters == 0
    # 8 DOFs: exact arithmetic ends in <= 8 steps; the solve reaches the dense solution
    A = brute.dense_matrix(1, 1, 1, 1, ref.V, 1.0)
    rs = m.cg(1.0, b, x, max_iter=64, fixed_iters=False, rtol=1e-14)
    assert rs.status == hb.HB_OK
    xs = np.linalg.solve(A, host(b))
    assert relerr(host(x), xs) <= 1e-12


def load_history(name):
    """Stored oracle history: (||r_j|| compensated, bar_j), written by tests/golden/make_cg_history.py."""
    rows = np.array([[float(v) for v in l.split()] for l in open(golden_path(name))
                     if l.strip() and not l.startswith("#")])
    return rows[:, 1], rows[:, 3]


def test_cg_large_config():
    """32^3 affine, N=7, 100 fixed iterations: every residual against the oracle's
    history (stored by a script that calls only the oracle) within the envelope of
    tests/cg_envelope.py; the recursive residual at the end against the oracle's
    true residual of the GPU iterate."""
    c = inputs.PLAIN_LARGE
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    say("[case] large config CG")
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    x = torch.empty_like(b)
    res = m.cg(c.lam, b, x, max_iter=c.iters, fixed_iters=True)
    assert res.status == hb.HB_OK and res.iters == c.iters
    h = np.array(res.history)
    href, bar = load_history("cg_history_box32_N7.txt")
    assert len(href) == c.iters + 1
    ratio = compare_history(h, href, bar)
    say(f"history ratio to bar (100 iterations): {ratio:.3f}")
    assert ratio <= 1.0
    # recursive residual after 100 iterations agrees with the true one
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    bh = oracle.rhs(m.NG, c.rhs_seed)
    assert np.array_equal(host(b), bh)
    rtrue = np.linalg.norm(bh - ref.ax(host(x), c.lam))
    assert abs(rtrue - h[-1]) <= 1e-9 * h[0]
    m.close()


def test_stream_probe():
    n = 1 << 20
    inp = torch.randn(8 * n, dtype=torch.float64, device=DEV)
    out = torch.empty(n, dtype=torch.float64, device=DEV)
    hb.stream_probe(inp, out)
    ref = inp.view(8, n).sum(0)
    assert torch.allclose(out, ref, rtol=1e-14, atol=1e-14)
