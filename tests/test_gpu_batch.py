"""Batched solves of independent problems (hb_batch_solve) on the GPU.

A batch runs the same algorithm per problem as the single-problem solver; only
the reduction order of the vector kernels differs (contiguous chunks instead
of a grid-stride sweep), so FP64 batched results agree with one-by-one solves
to rounding and with the oracle within the residual-history envelope.
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

# small uneven problems: every degree class the batched workload uses, plus a
# single element and a ragged operator tail
SMALL = [inputs.BoxCase("b0", 1, 1, 1, 3, 0.0, 1, 11), inputs.BoxCase("b1", 4, 4, 4, 3, 0.05, 1, 2),
         inputs.BoxCase("b2", 3, 2, 2, 5, 0.05, 3, 13), inputs.BoxCase("b3", 2, 3, 2, 7, 0.05, 4, 14),
         inputs.BoxCase("b4", 2, 2, 2, 9, 0.05, 5, 15), inputs.BoxCase("b5", 5, 3, 1, 1, 0.0, 6, 16)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def setup(cases, fp32=False):
    ms, bs, xs = [], [], []
    for c in cases:
        m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=fp32)
        b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
        hb.rhs_uniform(b, c.rhs_seed)
        ms.append(m)
        bs.append(b)
        xs.append(torch.full_like(b, float("nan")))
    return ms, bs, xs


def test_batch_fixed_iterations_match_single_solves():
    say("[case] batch FP64 fixed 60 iterations vs one-by-one")
    ms, bs, xs = setup(SMALL)
    st, res = hb.batch_solve(ms, [c.lam for c in SMALL], bs, xs, max_iter=60, fixed_iters=True)
    assert st == hb.HB_OK
    for c, m, b, x, r in zip(SMALL, ms, bs, xs, res):
        x1 = torch.empty_like(b)
        r1 = m.cg(c.lam, b, x1, max_iter=60, fixed_iters=True)
        assert r.iters == r1.iters and r.status == r1.status, c.name
        xb, xs1 = host(x), host(x1)
        assert np.linalg.norm(xb - xs1) <= 1e-9 * np.linalg.norm(xs1), c.name
        assert r.res == pytest.approx(r1.res, rel=1e-8)


def test_batch_fp64_matches_oracle_history_end():
    """Each batched FP64 problem's final residual after 100 iterations agrees with the
    oracle's residual history (same envelope as the one-problem parity test)."""
    say("[case] batch FP64 vs oracle")
    ms, bs, xs = setup(SMALL)
    st, res = hb.batch_solve(ms, [c.lam for c in SMALL], bs, xs, max_iter=100, fixed_iters=True)
    assert st == hb.HB_OK
    for c, r in zip(SMALL, res):
        ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
        bh = oracle.rhs(ref.NG, c.rhs_seed)
        href, bar = history_bar(ref, bh, c.lam, 100)
        k = r.iters
        got = np.array(href)
        got[k] = r.res
        assert compare_history(got[: k + 1], href[: k + 1], bar[: k + 1]) <= 1.0, c.name


def test_batch_graph_replay_matches_single_solves():
    """Segments replayed from captured graphs (16 iterations, which does not
    divide the 60: the device stops each problem at its cap) give the one-by-one
    solves' results."""
    say("[case] batch FP64 fixed 60 iterations, graph_k=16, vs one-by-one")
    ms, bs, xs = setup(SMALL)
    st, res = hb.batch_solve(ms, [c.lam for c in SMALL], bs, xs, max_iter=60, fixed_iters=True, graph_k=16)
    assert st == hb.HB_OK
    for c, m, b, x, r in zip(SMALL, ms, bs, xs, res):
        x1 = torch.empty_like(b)
        r1 = m.cg(c.lam, b, x1, max_iter=60, fixed_iters=True)
        assert r.iters == r1.iters == 60 and r.status == r1.status, c.name
        xb, xs1 = host(x), host(x1)
        assert np.linalg.norm(xb - xs1) <= 1e-9 * np.linalg.norm(xs1), c.name
        assert r.res == pytest.approx(r1.res, rel=1e-8)


@pytest.mark.parametrize("prec,graph_k", [(hb.PREC_FP64, 0), (hb.PREC_FP32_RR, 0), (hb.PREC_FP64, 10),
                                          (hb.PREC_FP32_RR, 10)])
def test_batch_tolerance_solves(prec, graph_k):
    say(f"[case] batch tolerance prec={prec} graph_k={graph_k}")
    ms, bs, xs = setup(SMALL, fp32=True)
    st, res = hb.batch_solve(ms, [c.lam for c in SMALL], bs, xs, max_iter=5000, rtol=1e-9, prec=prec,
                             check_every=10, graph_k=graph_k)
    assert st == hb.HB_OK, [r.status for r in res]
    for c, x, r in zip(SMALL, xs, res):
        ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
        bh = oracle.rhs(ref.NG, c.rhs_seed)
        tr = np.linalg.norm(bh - ref.ax(host(x), c.lam)) / np.linalg.norm(bh)
        say(f"{c.name}: iters {r.iters} outer {r.outer_iters} true residual {tr:.2e}")
        assert tr <= 1.2e-9, c.name
        # the same problem solved alone
        m1 = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=True)
        x1 = torch.empty_like(x)
        b1 = torch.empty_like(x)
        hb.rhs_uniform(b1, c.rhs_seed)
        r1 = m1.cg(c.lam, b1, x1, max_iter=5000, fixed_iters=False, rtol=1e-9, prec=prec, check_every=10)
        assert r1.status == hb.HB_OK
        # the two solutions agree to the tolerance both were solved to: ||A (x_batch - x_alone)|| <= 2 tol ||b||
        d = ref.ax(host(x) - host(x1), c.lam)
        assert np.linalg.norm(d) <= 2.2e-9 * np.linalg.norm(bh), c.name
        if prec == hb.PREC_FP64:
            assert abs(r.iters - r1.iters) <= 1, (c.name, r.iters, r1.iters)
        else:
            # FP32 atomic assembly sums in a run-dependent order, so the replacement points and
            # the iteration count vary between runs
            assert abs(r.iters - r1.iters) <= 0.2 * r1.iters + 5, (c.name, r.iters, r1.iters)


def test_batch_argument_errors():
    ms, bs, xs = setup(SMALL[:2])
    with pytest.raises(hb.HbError):  # the same mesh twice
        hb.batch_solve([ms[0], ms[0]], [1.0, 1.0], [bs[0], bs[0].clone()], [xs[0], xs[0].clone()])
    with pytest.raises(hb.HbError):  # no FP32 data
        hb.batch_solve(ms, [1.0, 1.0], bs, xs, prec=hb.PREC_FP32_RR)
    with pytest.raises(hb.HbError):
        hb.batch_solve(ms, [1.0, -1.0], bs, xs)
    for k in (-1, 4097):
        with pytest.raises(hb.HbError):
            hb.batch_solve(ms, [1.0, 1.0], bs, xs, graph_k=k)
    st, res = hb.batch_solve([], [], [], [])
    assert st == hb.HB_OK and res == []


def test_batched_workload_full_size():
    """The 64-problem batched workload at its full size, solved as the benchmark
    solves it (FP32 operator with FP64 residual replacement, to 1e-8): every
    problem's true residual, computed with the oracle's FP64 operator, meets the
    tolerance."""
    cases = inputs.batched_cases()
    say(f"[case] batched workload, {len(cases)} problems, FP32 RR to 1e-8")
    ms, bs, xs = setup(cases, fp32=True)
    st, res = hb.batch_solve(ms, [c.lam for c in cases], bs, xs, max_iter=100000, rtol=1e-8,
                             prec=hb.PREC_FP32_RR)
    assert st == hb.HB_OK, [r.status for r in res]
    for m in ms:
        m.close()
    worst = 0.0
    for i, (c, x, r) in enumerate(zip(cases, xs, res)):
        ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
        bh = oracle.rhs(ref.NG, c.rhs_seed)
        tr = np.linalg.norm(bh - ref.ax(host(x), c.lam)) / np.linalg.norm(bh)
        del ref
        worst = max(worst, tr)
        if i % 8 == 0:
            say(f"{i}: {c.name} iters {r.iters} replacements {r.outer_iters} true residual {tr:.2e}")
        assert r.status == hb.HB_OK and tr <= 1.2e-8, (c.name, r, tr)
    say(f"worst true residual {worst:.2e}")
