"""CG iterations replayed from a captured HIP graph (hb_cg_opts.graph_k).

A graph replays exactly the kernels of the plain launch path, so the results
obey the same bars: the residual history within the oracle envelope, the same
iteration count (the device state stops the solve; replays past the stop do
nothing, so graph lengths that do not divide the iteration count are exact),
and every replay of a cached graph agrees with the plain launch path, with
eager work on the same stream between replays.
"""
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


@pytest.mark.parametrize("k", [1, 7, 100])
def test_graph_fixed_iterations_match_oracle_and_plain(k):
    c = inputs.PLAIN_SMALL
    say(f"[case] graph_k={k} small config 100 iterations")
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    bh = oracle.rhs(m.NG, c.rhs_seed)
    href, bar = history_bar(ref, bh, c.lam, c.iters)
    x_plain = torch.empty_like(b)
    r_plain = m.cg(c.lam, b, x_plain, max_iter=c.iters, fixed_iters=True)
    x = torch.empty_like(b)
    y = torch.empty_like(b)
    for rep in range(3):
        x.fill_(float("nan"))
        res = m.cg(c.lam, b, x, max_iter=c.iters, fixed_iters=True, graph_k=k)
        assert res.status == hb.HB_OK and res.iters == c.iters, (rep, res)
        ratio = compare_history(res.history, href, bar)
        say(f"replay {rep}: history ratio to bar {ratio:.3f}")
        assert ratio <= 1.0
        assert relerr(host(x), host(x_plain)) <= 1e-9
        assert res.res == pytest.approx(r_plain.res, rel=1e-8)
        # eager work on the same stream between replays
        m.ax(c.lam, x, y)
        assert relerr(host(y), ref.ax(host(x), c.lam)) <= 1e-12
    m.close()


def test_graph_tolerance_mode_stops_where_plain_stops():
    say("[case] graph_k=10 tolerance mode")
    m = hb.Mesh(3, 3, 3, 4, jitter=0.05, seed=5)
    ref = oracle.Mesh(3, 3, 3, 4, jitter=0.05, seed=5)
    bh = oracle.rhs(m.NG, 11)
    b = torch.as_tensor(bh, device=DEV)
    x = torch.zeros_like(b)
    out = ref.cg(bh, 1.0, max_iter=2000, rtol=1e-8)
    for check_every in (10, 25):
        res = m.cg(1.0, b, x, max_iter=2000, fixed_iters=False, rtol=1e-8, check_every=check_every, graph_k=10)
        assert res.status == hb.HB_OK
        assert abs(res.iters - out["iters"]) <= 1
        assert res.res <= 1e-8 * res.bnorm
        assert np.linalg.norm(bh - ref.ax(host(x), 1.0)) <= 2e-8 * np.linalg.norm(bh)
    # an iteration cap inside a graph replay: NOT_CONVERGED exactly at the cap
    res = m.cg(1.0, b, x, max_iter=13, fixed_iters=False, rtol=1e-12, graph_k=10)
    assert res.status == hb.HB_ERR_NOT_CONVERGED and res.iters == 13 and len(res.history) == 14
    m.close()


@pytest.mark.parametrize("prec", [hb.PREC_FP32_RR, hb.PREC_FP32_IR])
def test_graph_mixed_precision(prec):
    c = inputs.PLAIN_SMALL
    say(f"[case] graph_k=5 mixed prec={prec}")
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=True)
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    bh = oracle.rhs(m.NG, c.rhs_seed)
    x = torch.empty_like(b)
    res = m.cg(c.lam, b, x, max_iter=5000, fixed_iters=False, rtol=1e-10, prec=prec, graph_k=5)
    assert res.status == hb.HB_OK
    assert np.linalg.norm(bh - ref.ax(host(x), c.lam)) <= 1.2e-10 * np.linalg.norm(bh)
    m.close()


def test_graph_argument_errors():
    m = hb.Mesh(2, 2, 2, 3)
    b = torch.ones(m.NG, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    for k in (-1, 4097):
        with pytest.raises(hb.HbError) as e:
            m.cg(1.0, b, x, max_iter=10, fixed_iters=True, graph_k=k)
        assert e.value.status == hb.HB_ERR_INVALID_ARG
    m.close()
