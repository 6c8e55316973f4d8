"""The two-phase operator on the GPU (HB_MESH_GATHER: the element kernel writes
the local vector y_L, then Z^T is applied as a gather over CSR rows), against
the oracle through the C ABI: y = A x and y += A x within 1e-12 for every
degree on ragged boxes (plain and Dirichlet, both mass kinds), bit-identical
repeated applications and CG solves, CG and Jacobi-PCG residual histories
within the oracle envelope (plain launches and graph replay), the 32^3 N=7
workload in full, and the argument checks."""
import ctypes
import sys

import numpy as np
import pytest

import inputs
import oracle
from cg_envelope import compare_history, history_bar

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2202_12477_amd as hb  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [(5, 3, 2, 1), (4, 2, 3, 2), (3, 3, 2, 3), (4, 2, 2, 4), (2, 3, 2, 5), (3, 2, 2, 6), (3, 2, 2, 7),
         (2, 2, 1, 8), (2, 1, 2, 9), (1, 2, 1, 10), (2, 1, 1, 11), (1, 1, 2, 12), (1, 2, 1, 13), (1, 1, 1, 14),
         (2, 1, 1, 15)]


@pytest.mark.parametrize("nx,ny,nz,N", CASES)
@pytest.mark.parametrize("dirichlet", [False, True])
def test_two_phase_ax_matches_oracle(nx, ny, nz, N, dirichlet):
    say(f"[case] two-phase Ax {nx}x{ny}x{nz} N={N} dirichlet={dirichlet}")
    m = hb.Mesh(nx, ny, nz, N, jitter=0.05, seed=N, dirichlet=dirichlet, gather=True)
    ref = oracle.Mesh(nx, ny, nz, N, jitter=0.05, seed=N, dirichlet=dirichlet)
    assert m.NG == ref.NG
    x = inputs.random_vector(m.NG, 70 + N)
    yr = ref.ax(x, 1.3)
    xd = torch.as_tensor(x, device=DEV)
    y = torch.full_like(xd, float("nan"))  # overwritten, never read
    m.ax(1.3, xd, y)
    e = relerr(host(y), yr)
    y0 = torch.as_tensor(inputs.random_vector(m.NG, 90 + N), device=DEV)
    y2 = y0.clone()
    m.ax_add(1.3, xd, y2)
    e_add = relerr(host(y2) - host(y0), yr)
    y3 = torch.empty_like(xd)
    m.ax(1.3, xd, y3)
    say(f"  y = Ax {e:.2e}; y += Ax {e_add:.2e}")
    assert e <= 1e-12 and e_add <= 1e-12
    assert torch.equal(y, y3)  # the gather sums in a fixed order
    m.close()


@pytest.mark.parametrize("mass", [hb.MASS_GWJ, hb.MASS_INVDEG])
def test_two_phase_mass_kinds(mass):
    m = hb.Mesh(3, 3, 3, 4, jitter=0.05, seed=2, mass=mass, gather=True)
    ref = oracle.Mesh(3, 3, 3, 4, jitter=0.05, seed=2, mass=mass)
    x = inputs.random_vector(m.NG, 9)
    y = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    m.ax(0.9, torch.as_tensor(x, device=DEV), y)
    assert relerr(host(y), ref.ax(x, 0.9)) <= 1e-12


@pytest.mark.parametrize("graph_k", [0, 9])
def test_two_phase_cg_history_and_determinism(graph_k):
    """The small configuration, 100 fixed iterations: the residual history within
    the oracle envelope, and a second solve bit-identical to the first."""
    c = inputs.PLAIN_SMALL
    say(f"[case] two-phase CG, small config, graph_k={graph_k}")
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, gather=True)
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    bh = oracle.rhs(m.NG, c.rhs_seed)
    x1, x2 = torch.empty_like(b), torch.empty_like(b)
    r1 = m.cg(c.lam, b, x1, max_iter=100, fixed_iters=True, graph_k=graph_k)
    r2 = m.cg(c.lam, b, x2, max_iter=100, fixed_iters=True, graph_k=graph_k)
    assert r1.status == hb.HB_OK and r1.iters == 100
    href, bar = history_bar(ref, bh, c.lam, 100)
    ratio = compare_history(r1.history, href, bar)
    say(f"  history ratio to bar {ratio:.3f}")
    assert ratio <= 1.0
    assert r1.history == r2.history
    assert torch.equal(x1, x2)


def test_two_phase_pcg_and_dirichlet_tolerance():
    m = hb.Mesh(4, 3, 3, 5, jitter=0.1, seed=3, dirichlet=True, gather=True)
    ref = oracle.Mesh(4, 3, 3, 5, jitter=0.1, seed=3, dirichlet=True)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, 17)
    bh = oracle.rhs(m.NG, 17)
    for pc in (hb.PRECOND_NONE, hb.PRECOND_JACOBI):
        x = torch.empty_like(b)
        res = m.cg(1.0, b, x, max_iter=5000, fixed_iters=False, rtol=1e-10, precond=pc)
        assert res.status == hb.HB_OK, res
        tr = np.linalg.norm(bh - ref.ax(host(x), 1.0)) / np.linalg.norm(bh)
        o = (ref.pcg if pc else ref.cg)(bh, 1.0, max_iter=5000, rtol=1e-10)
        say(f"  precond {pc}: {res.iters} iterations (oracle {o['iters']}), true residual {tr:.2e}")
        assert tr <= 1.2e-10 and abs(res.iters - o["iters"]) <= 2


def test_two_phase_full_workload():
    """The 32^3 N=7 affine box (11.4M DOFs) in the launch configuration the
    benchmark times: the whole vector against the oracle, and against the fused operator."""
    c = inputs.PLAIN_LARGE
    say("[case] two-phase Ax at 32^3 N=7")
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, gather=True)
    f = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    y, yf = torch.empty_like(b), torch.empty_like(b)
    m.ax(c.lam, b, y)
    f.ax(c.lam, b, yf)
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    yr = ref.ax(oracle.rhs(m.NG, c.rhs_seed), c.lam)
    e, ef = relerr(host(y), yr), relerr(host(y), host(yf))
    say(f"  vs oracle {e:.2e}, vs fused {ef:.2e}")
    assert e <= 1e-12 and ef <= 1e-12
    m.close()
    f.close()


def test_two_phase_argument_checks():
    m = hb.Mesh(2, 2, 2, 3, gather=True)
    b = torch.ones(m.NG, dtype=torch.float64, device=DEV)
    x = torch.empty_like(b)
    with pytest.raises(hb.HbError):
        hb.batch_solve([m], [1.0], [b], [x], max_iter=5)
    with pytest.raises(hb.HbError):
        m.cg(1.0, b, x, max_iter=50, fixed_iters=False, rtol=1e-8, prec=hb.PREC_FP32_RR)
    with pytest.raises(hb.HbError):
        hb.Mesh(2, 2, 2, 3, gather=True, fp32=True)
    eng = hb.Engine(1 << 28, max_slots=2, prec=hb.PREC_FP64, iters_per_step=10)
    d = hb._MeshDesc(2, 2, 2, 3, 0.0, 0, hb.MASS_GWJ, hb.MESH_GATHER)
    t = ctypes.c_uint64()
    assert hb.lib().hb_engine_submit(eng._h, ctypes.byref(d), 1.0, 1, 1e-8, ctypes.byref(t)) == \
        hb.HB_ERR_INVALID_ARG
    eng.close()
    m.close()
