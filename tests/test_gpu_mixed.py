"""FP32 operator and FP64 iterative refinement on the GPU, through the C ABI.

The paper is FP64 throughout, so the FP32 operator's exact values have no
reference ("parity unpinned"); it is checked against the FP64 oracle with a
bar derived from its arithmetic: each output sums about 3(N+1)+8 FP32 products
of inputs already rounded once to FP32, so its relative error is a small
multiple of (3(N+1)+8) u32 (u32 = 2^-24) times the cancellation in A x for a
random x; 2e-5 covers N <= 15 with margin, and the test also requires the
error to be clearly above FP64 rounding (it must really be FP32).
The refined solution is checked the way the solver promises: the oracle's
FP64 operator gives ||b - A x|| <= rtol ||b||.
"""
import sys

import numpy as np
import pytest

import inputs
import oracle

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
    return t.cpu().numpy().astype(np.float64)


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_ax_f32_error_per_degree(N):
    n = 3 if N <= 6 else 2
    say(f"[case] ax_f32 N={N} box {n}x{n}x{n}")
    m = hb.Mesh(n, n, n, N, jitter=0.05, seed=20 + N, fp32=True)
    ref = oracle.Mesh(n, n, n, N, jitter=0.05, seed=20 + N)
    x = inputs.random_vector(m.NG, 40 + N)
    y = torch.full((m.NG,), float("nan"), dtype=torch.float32, device=DEV)
    m.ax_f32(1.0, dev(x), y)
    err = relerr(host(y), ref.ax(x, 1.0))
    say(f"FP32 operator relative error N={N}: {err:.3e}")
    assert 1e-9 < err <= 2e-5


def test_ax_f32_needs_fp32_mesh():
    m = hb.Mesh(2, 2, 2, 3)
    x = torch.zeros(m.NG, dtype=torch.float64, device=DEV)
    y = torch.zeros(m.NG, dtype=torch.float32, device=DEV)
    with pytest.raises(hb.HbError) as e:
        m.ax_f32(1.0, x, y)
    assert e.value.status == hb.HB_ERR_INVALID_ARG


MIXED = [hb.PREC_FP32_IR, hb.PREC_FP32_RR]


def solve_mixed(case, rtol, prec, **kw):
    m = hb.Mesh(case.nx, case.ny, case.nz, case.N, jitter=case.jitter, seed=case.mesh_seed, fp32=True)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, case.rhs_seed)
    x = torch.empty_like(b)
    res = m.cg(case.lam, b, x, max_iter=20000, fixed_iters=False, rtol=rtol, prec=prec, **kw)
    return m, b, x, res


def oracle_true_residual(case, x):
    ref = oracle.Mesh(case.nx, case.ny, case.nz, case.N, jitter=case.jitter, seed=case.mesh_seed)
    bh = oracle.rhs(ref.NG, case.rhs_seed)
    return np.linalg.norm(bh - ref.ax(x, case.lam)) / np.linalg.norm(bh)


@pytest.mark.parametrize("prec", MIXED)
def test_refinement_small_config(prec):
    c = inputs.PLAIN_SMALL
    say(f"[case] mixed prec={prec} small config to 1e-10")
    m, b, x, res = solve_mixed(c, 1e-10, prec)
    say(f"outer {res.outer_iters} inner {res.iters} fp64 {res.fp64_iters} res/b {res.res / res.bnorm:.2e}")
    assert res.status == hb.HB_OK and res.fp64_iters == 0 and res.outer_iters >= 2
    assert res.res <= 1e-10 * res.bnorm
    assert oracle_true_residual(c, host(x)) <= 1.2e-10
    # the refinement history is the true residual per step, decreasing
    h = np.array(res.history)
    assert len(h) == res.outer_iters + 1 and np.all(np.diff(h) < 0)
    # FP64 CG on the same problem reaches the same solution
    x64 = torch.empty_like(b)
    r64 = m.cg(c.lam, b, x64, max_iter=20000, fixed_iters=False, rtol=1e-12)
    assert r64.status == hb.HB_OK
    assert relerr(host(x), host(x64)) <= 1e-6


@pytest.mark.parametrize("prec", MIXED)
def test_refinement_falls_back_to_fp64_when_stalled(prec):
    """An inner tolerance of 0.9 cannot halve the residual per step: the solver must
    notice the stall and finish with the FP64 operator."""
    c = inputs.PLAIN_SMALL
    say(f"[case] mixed prec={prec} forced stall")
    m, b, x, res = solve_mixed(c, 1e-9, prec, inner_rtol=0.9)
    assert res.status == hb.HB_OK and res.fp64_iters > 0
    assert oracle_true_residual(c, host(x)) <= 1.2e-9


def test_refinement_argument_errors():
    m = hb.Mesh(2, 2, 2, 3)  # no FP32 data
    b = torch.ones(m.NG, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    with pytest.raises(hb.HbError) as e:
        m.cg(1.0, b, x, max_iter=10, fixed_iters=False, rtol=1e-6, prec=hb.PREC_FP32_IR)
    assert e.value.status == hb.HB_ERR_INVALID_ARG
    m2 = hb.Mesh(2, 2, 2, 3, fp32=True)
    with pytest.raises(hb.HbError) as e:
        m2.cg(1.0, b, x, max_iter=10, fixed_iters=True, prec=hb.PREC_FP32_IR)
    assert e.value.status == hb.HB_ERR_INVALID_ARG


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_refinement_order_sweep(N):
    """The order sweep at every degree: the sweep mesh (about 2^24 local nodes,
    jittered) solved to 1e-10 by restarted refinement and by residual replacement,
    both with the FP32 operator; the oracle's FP64 operator confirms each true
    residual (one oracle mesh per degree serves both solves)."""
    c = inputs.order_sweep_case(N)
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=True)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    xs = {}
    for prec in MIXED:
        say(f"[case] mixed prec={prec} order sweep N={N} n={c.nx}")
        x = torch.empty_like(b)
        res = m.cg(c.lam, b, x, max_iter=40000, fixed_iters=False, rtol=1e-10, prec=prec)
        say(f"N={N} prec={prec}: outer {res.outer_iters} inner {res.iters} fp64 {res.fp64_iters} "
            f"res/b {res.res / res.bnorm:.2e}")
        assert res.status == hb.HB_OK
        assert res.res <= 1e-10 * res.bnorm
        xs[prec] = host(x)
    m.close()
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    bh = oracle.rhs(ref.NG, c.rhs_seed)
    assert np.array_equal(host(b), bh)
    for prec, x in xs.items():
        tr = np.linalg.norm(bh - ref.ax(x, c.lam)) / np.linalg.norm(bh)
        say(f"N={N} prec={prec}: oracle FP64 true residual {tr:.3e}")
        assert tr <= 1.2e-10
