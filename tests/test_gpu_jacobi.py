"""Jacobi-preconditioned CG on the GPU (hb_cg_solve with HB_PRECOND_JACOBI)
against the oracle's preconditioned CG through the C ABI: fixed-iteration
residual histories within the envelope of the oracle's two summation orders
(plain box, Dirichlet box, graph replay), tolerance solves checked by their
true residual under the oracle's FP64 operator, fewer iterations than the
unpreconditioned solve on a deformed mesh, batched PCG over uneven problems
(hb_batch_solve, with and without graph replay), and the argument checks."""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def pcg_bar(ref, b, lam, iters):
    """(oracle residual history, per-iteration relative bar): 1e-10, or 10x the
    spread between the oracle's compensated and plain dot products where that is larger."""
    h = ref.pcg(b, lam, fixed_iters=iters, compensated=True)["res"]
    alt = ref.pcg(b, lam, fixed_iters=iters, compensated=False)["res"]
    return h, np.maximum(1e-10, 10.0 * np.abs(h - alt) / np.abs(h))


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def ratio_to_bar(got, ref, bar):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    live = ref / ref[0] > 1e-13
    return float(np.max(np.abs(got - ref)[live] / (np.abs(ref[live]) * bar[live])))


def setup(nx, ny, nz, N, jitter, seed, rhs_seed, dirichlet=False):
    m = hb.Mesh(nx, ny, nz, N, jitter=jitter, seed=seed, dirichlet=dirichlet)
    ref = oracle.Mesh(nx, ny, nz, N, jitter=jitter, seed=seed, dirichlet=dirichlet)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, rhs_seed)
    bh = oracle.rhs(m.NG, rhs_seed)
    assert np.array_equal(host(b), bh)
    return m, ref, b, bh


@pytest.mark.parametrize("dirichlet,graph_k", [(False, 0), (True, 0), (False, 8), (True, 7)])
def test_pcg_history_matches_oracle(dirichlet, graph_k):
    """60 fixed iterations on the small configuration's jittered box (4^3, N=3,
    and a 3x2x2 N=6 box whose element rows fall in ragged vector blocks)."""
    for (nx, ny, nz, N) in [(4, 4, 4, 3), (3, 2, 2, 6)]:
        say(f"[case] PCG history {nx}x{ny}x{nz} N={N} dirichlet={dirichlet} graph_k={graph_k}")
        m, ref, b, bh = setup(nx, ny, nz, N, 0.1, 7, 11, dirichlet)
        x = torch.empty_like(b)
        res = m.cg(1.0, b, x, max_iter=60, fixed_iters=True, precond=hb.PRECOND_JACOBI, graph_k=graph_k)
        assert res.status == hb.HB_OK and res.iters == 60, res
        href, bar = pcg_bar(ref, bh, 1.0, 60)
        r = ratio_to_bar(res.history, href, bar)
        say(f"  history ratio to bar {r:.3f}; ||r_60||/||r_0|| {href[-1] / href[0]:.2e}")
        assert r <= 1.0
        assert res.res0 == pytest.approx(np.linalg.norm(bh), rel=1e-13)
        xo = ref.pcg(bh, 1.0, fixed_iters=60)["x"]
        ex = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
        say(f"  solution vs oracle {ex:.2e}")
        assert ex <= 1e-9
        m.close()


def test_pcg_lambda_change_recomputes_the_diagonal():
    """The preconditioner is kept with the mesh per lambda: a second solve at
    another lambda (and a third back at the first) follows the oracle."""
    m, ref, b, bh = setup(3, 3, 2, 5, 0.1, 4, 5)
    for lam in (1.0, 0.05, 1.0):
        say(f"[case] PCG lambda {lam}")
        x = torch.empty_like(b)
        res = m.cg(lam, b, x, max_iter=40, fixed_iters=True, precond=hb.PRECOND_JACOBI)
        href, bar = pcg_bar(ref, bh, lam, 40)
        r = ratio_to_bar(res.history, href, bar)
        say(f"  history ratio to bar {r:.3f}")
        assert r <= 1.0
    m.close()


@pytest.mark.parametrize("dirichlet", [False, True])
def test_pcg_tolerance_solve_and_iteration_saving(dirichlet):
    """A deformed 4x3x3 N=7 box: PCG to 1e-10 reaches the tolerance on the true
    residual, in no more iterations than the oracle's PCG (+2), and in fewer than plain CG."""
    say(f"[case] PCG tolerance solve dirichlet={dirichlet}")
    m, ref, b, bh = setup(4, 3, 3, 7, 0.2, 9, 21, dirichlet)
    x = torch.empty_like(b)
    pres = m.cg(1.0, b, x, max_iter=5000, fixed_iters=False, rtol=1e-10, precond=hb.PRECOND_JACOBI)
    assert pres.status == hb.HB_OK, pres
    tr = np.linalg.norm(bh - ref.ax(host(x), 1.0)) / np.linalg.norm(bh)
    o = ref.pcg(bh, 1.0, max_iter=5000, rtol=1e-10)
    x2 = torch.empty_like(b)
    cres = m.cg(1.0, b, x2, max_iter=5000, fixed_iters=False, rtol=1e-10)
    assert cres.status == hb.HB_OK, cres
    say(f"  PCG {pres.iters} iters (oracle {o['iters']}), CG {cres.iters}; true residual {tr:.2e}")
    assert tr <= 1.2e-10
    assert abs(pres.iters - o["iters"]) <= 2
    assert pres.iters < cres.iters
    assert pres.res <= 1e-10 * pres.bnorm
    m.close()


def test_pcg_argument_checks():
    m = hb.Mesh(2, 2, 2, 3, fp32=True)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, 3)
    x = torch.empty_like(b)
    with pytest.raises(hb.HbError):
        m.cg(1.0, b, x, max_iter=5, precond=7)
    with pytest.raises(hb.HbError):
        m.cg(1.0, b, x, max_iter=5, precond=-1)
    with pytest.raises(hb.HbError):
        hb.batch_solve([m], [1.0], [b], [x], max_iter=50, rtol=1e-8, prec=hb.PREC_FP32_IR,
                       precond=hb.PRECOND_JACOBI)
    with pytest.raises(hb.HbError):
        hb.batch_solve([m], [1.0], [b], [x], max_iter=5, precond=3)
    # an unpreconditioned solve after a preconditioned one is plain CG again
    res = m.cg(1.0, b, x, max_iter=10, precond=hb.PRECOND_JACOBI)
    assert res.status == hb.HB_OK
    ref = oracle.Mesh(2, 2, 2, 3)
    plain = m.cg(1.0, b, x, max_iter=10)
    h = ref.cg(oracle.rhs(ref.NG, 3), 1.0, fixed_iters=10)["res"]
    assert np.allclose(plain.history, h, rtol=1e-9, atol=0)
    m.close()


@pytest.mark.parametrize("graph_k", [0, 6])
def test_batched_pcg(graph_k):
    """hb_batch_solve with the Jacobi preconditioner over uneven problems (plain
    and Dirichlet boxes, N = 3..9): each reaches 1e-10 on its true residual in the
    oracle's PCG iteration count (+-2), and 40 fixed iterations match the
    one-problem PCG solution."""
    say(f"[case] batched PCG graph_k={graph_k}")
    shapes = [(3, 3, 3, 3, False), (2, 3, 2, 7, True), (2, 2, 2, 9, False), (4, 2, 3, 5, True)]
    ms, refs, bs, bhs = [], [], [], []
    for i, (nx, ny, nz, N, d) in enumerate(shapes):
        m, ref, b, bh = setup(nx, ny, nz, N, 0.15, 20 + i, 30 + i, d)
        ms.append(m), refs.append(ref), bs.append(b), bhs.append(bh)
    lams = [1.0, 0.5, 1.0, 2.0]
    xs = [torch.empty_like(b) for b in bs]
    st, res = hb.batch_solve(ms, lams, bs, xs, max_iter=5000, rtol=1e-10, precond=hb.PRECOND_JACOBI, graph_k=graph_k)
    assert st == hb.HB_OK, [r.status for r in res]
    for i in range(len(shapes)):
        o = refs[i].pcg(bhs[i], lams[i], max_iter=5000, rtol=1e-10)
        tr = np.linalg.norm(bhs[i] - refs[i].ax(host(xs[i]), lams[i])) / np.linalg.norm(bhs[i])
        say(f"  problem {i}: {res[i].iters} iterations (oracle {o['iters']}), true residual {tr:.2e}")
        assert abs(res[i].iters - o["iters"]) <= 2 and tr <= 1.2e-10
        assert res[i].res0 == pytest.approx(np.linalg.norm(bhs[i]), rel=1e-13)
        assert res[i].res <= 1e-10 * res[i].bnorm
    xs = [torch.empty_like(b) for b in bs]
    st, res = hb.batch_solve(ms, lams, bs, xs, max_iter=40, fixed_iters=True, precond=hb.PRECOND_JACOBI,
                             graph_k=graph_k)
    assert st == hb.HB_OK and all(r.iters == 40 for r in res)
    for i, m in enumerate(ms):
        x1 = torch.empty_like(bs[i])
        m.cg(lams[i], bs[i], x1, max_iter=40, fixed_iters=True, precond=hb.PRECOND_JACOBI)
        ex = relerr(host(xs[i]), host(x1))
        xo = refs[i].pcg(bhs[i], lams[i], fixed_iters=40)["x"]
        eo = relerr(host(xs[i]), xo)
        say(f"  problem {i}: 40 iterations vs one-problem {ex:.2e}, vs oracle {eo:.2e}")
        assert ex <= 1e-9 and eo <= 1e-9
    for m in ms:
        m.close()


@pytest.mark.parametrize("graphs", [False, True])
def test_engine_pcg(graphs):
    """The serving engine with the Jacobi preconditioner (FP64, plain launches and
    graph replay of its steps): every request reaches its tolerance on the true
    residual in the oracle's PCG iteration count (+-2)."""
    say(f"[case] engine PCG graphs={graphs}")
    reqs = [(3, 3, 2, 5, False, 41), (2, 2, 3, 7, True, 42), (4, 3, 3, 3, True, 43)]
    eng = hb.Engine(1 << 30, max_slots=2, prec=hb.PREC_FP64, iters_per_step=15, precond=hb.PRECOND_JACOBI,
                    graphs=graphs)
    tickets = {eng.submit(nx, ny, nz, N, jitter=0.15, seed=s, rhs_seed=s + 100, rtol=1e-10, dirichlet=d): i
               for i, (nx, ny, nz, N, d, s) in enumerate(reqs)}
    got = {}
    for _ in range(100000):
        if len(got) == len(reqs):
            break
        eng.step()
        for t, i in tickets.items():
            if i not in got:
                out = eng.poll(t)
                if out is not None:
                    got[i] = out
    eng.close()
    assert len(got) == len(reqs)
    for i, (nx, ny, nz, N, d, s) in enumerate(reqs):
        ref = oracle.Mesh(nx, ny, nz, N, jitter=0.15, seed=s, dirichlet=d)
        bh = oracle.rhs(ref.NG, s + 100)
        res, x = got[i]
        o = ref.pcg(bh, 1.0, max_iter=5000, rtol=1e-10)
        tr = np.linalg.norm(bh - ref.ax(x, 1.0)) / np.linalg.norm(bh)
        say(f"  request {i}: {res.iters} iterations (oracle {o['iters']}), true residual {tr:.2e}")
        assert res.status == hb.HB_OK and abs(res.iters - o["iters"]) <= 2 and tr <= 1.2e-10


@pytest.mark.parametrize("dirichlet", [False, True])
def test_pcg_with_fp32_operator_and_replacement(dirichlet):
    """Jacobi with the FP32 operator: FP64 refinement (inner solves preconditioned)
    and FP64 residual replacement (one problem, batched and served); every solve
    meets 1e-10 on the FP64 true residual (the oracle's operator), and the
    single solves take fewer iterations than without the preconditioner on the
    deformed box."""
    say(f"[case] PCG + FP32 residual replacement, dirichlet={dirichlet}")
    nx, ny, nz, N = 4, 3, 3, 7
    m = hb.Mesh(nx, ny, nz, N, jitter=0.2, seed=9, fp32=True, dirichlet=dirichlet)
    ref = oracle.Mesh(nx, ny, nz, N, jitter=0.2, seed=9, dirichlet=dirichlet)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, 21)
    bh = oracle.rhs(m.NG, 21)

    def true_res(x):
        return np.linalg.norm(bh - ref.ax(host(x), 1.0)) / np.linalg.norm(bh)

    xi = torch.empty_like(b)
    ires = m.cg(1.0, b, xi, max_iter=20000, fixed_iters=False, rtol=1e-10, prec=hb.PREC_FP32_IR,
                precond=hb.PRECOND_JACOBI)
    xi2 = torch.empty_like(b)
    ires0 = m.cg(1.0, b, xi2, max_iter=20000, fixed_iters=False, rtol=1e-10, prec=hb.PREC_FP32_IR)
    tri = true_res(xi)
    say(f"  refinement: PCG inner {ires.iters} iterations ({ires.outer_iters} outer), CG inner {ires0.iters}; "
        f"true residual {tri:.2e}")
    assert ires.status == hb.HB_OK and tri <= 1.2e-10 and ires.iters < ires0.iters
    x = torch.empty_like(b)
    pres = m.cg(1.0, b, x, max_iter=20000, fixed_iters=False, rtol=1e-10, prec=hb.PREC_FP32_RR,
                precond=hb.PRECOND_JACOBI)
    tr = true_res(x)
    x2 = torch.empty_like(b)
    cres = m.cg(1.0, b, x2, max_iter=20000, fixed_iters=False, rtol=1e-10, prec=hb.PREC_FP32_RR)
    o = ref.pcg(bh, 1.0, max_iter=5000, rtol=1e-10)
    say(f"  single: PCG-RR {pres.iters} iterations ({pres.outer_iters} replacements), CG-RR {cres.iters}, "
        f"oracle PCG {o['iters']}; true residual {tr:.2e}")
    assert pres.status == hb.HB_OK and tr <= 1.2e-10
    assert pres.iters < cres.iters
    assert pres.res0 == pytest.approx(np.linalg.norm(bh), rel=1e-13)
    xs = [torch.empty_like(b)]
    st, res = hb.batch_solve([m], [1.0], [b], xs, max_iter=20000, rtol=1e-10, prec=hb.PREC_FP32_RR,
                             precond=hb.PRECOND_JACOBI)
    trb = true_res(xs[0])
    say(f"  batched: {res[0].iters} iterations, true residual {trb:.2e}")
    assert st == hb.HB_OK and trb <= 1.2e-10
    assert res[0].res0 == pytest.approx(np.linalg.norm(bh), rel=1e-13)
    m.close()
    eng = hb.Engine(1 << 30, max_slots=2, prec=hb.PREC_FP32_RR, iters_per_step=15, precond=hb.PRECOND_JACOBI)
    t = eng.submit(nx, ny, nz, N, jitter=0.2, seed=9, rhs_seed=21, rtol=1e-10, dirichlet=dirichlet)
    out = None
    for _ in range(100000):
        eng.step()
        out = eng.poll(t)
        if out is not None:
            break
    eng.close()
    r, xe = out
    tre = np.linalg.norm(bh - ref.ax(xe, 1.0)) / np.linalg.norm(bh)
    say(f"  engine: {r.iters} iterations, true residual {tre:.2e}")
    assert r.status == hb.HB_OK and tre <= 1.2e-10
