"""The Dirichlet box on the GPU (HB_MESH_DIRICHLET: the boundary nodes of
[0,1]^3 carry no DOF, N_G = (nx N - 1)(ny N - 1)(nz N - 1), the setting of the
paper's experiments), against the oracle's Dirichlet mesh through the C ABI:
the map bit-exact, y = A x within 1e-12 under every tile schedule (element
walks, face merging and ragged tails included), CG residual histories within the
envelope, and the mixed-precision, batched and served solves to their
tolerance (true residual with the oracle's FP64 operator)."""
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
PRECS = (hb.PREC_FP64, hb.PREC_FP32_RR)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def legal(N):
    base = [0, 1, 2, 3] if (N + 1) ** 2 <= 64 else [0, 1, 4, 5]
    return base + ([8, 9] if (N + 1) ** 2 <= 128 else []) + ([21] if N >= 8 else []) + ([29] if 8 <= N <= 10 else [])


@pytest.fixture(autouse=True)
def restore_table():
    saved = {(N, p): hb.get_schedule(N, p) for N in range(1, 16) for p in PRECS}
    yield
    for (N, p), v in saved.items():
        hb.set_schedule(N, p, v)


# ragged tails for every block shape, boxes with an even number of elements per
# row (tile walks) and odd ones (plain order)
CASES = [(5, 3, 2, 1), (4, 2, 3, 2), (3, 3, 2, 3), (4, 2, 2, 4), (2, 3, 2, 5), (3, 2, 2, 6), (3, 2, 2, 7),
         (2, 2, 1, 8), (2, 1, 2, 9), (1, 2, 1, 10), (2, 1, 1, 11), (1, 1, 2, 12), (1, 2, 1, 13), (1, 1, 1, 14),
         (2, 1, 1, 15)]


@pytest.mark.parametrize("nx,ny,nz,N", CASES)
def test_dirichlet_ax_matches_oracle_under_every_schedule(nx, ny, nz, N):
    say(f"[case] Dirichlet {nx}x{ny}x{nz} N={N}")
    m = hb.Mesh(nx, ny, nz, N, jitter=0.05, seed=N, fp32=True, dirichlet=True)
    ref = oracle.Mesh(nx, ny, nz, N, jitter=0.05, seed=N, dirichlet=True)
    assert m.NG == ref.NG == (nx * N - 1) * (ny * N - 1) * (nz * N - 1)
    _, mp, _, _, _ = m.export()
    assert np.array_equal(mp.ravel().astype(np.int64), ref.map)
    x = inputs.random_vector(m.NG, 40 + N)
    yr = ref.ax(x, 1.3)
    xd = torch.as_tensor(x, device=DEV)
    for v in legal(N):
        hb.set_schedule(N, hb.PREC_FP64, v)
        hb.set_schedule(N, hb.PREC_FP32_RR, v)
        y = torch.empty_like(xd)
        m.ax(1.3, xd, y)
        y32 = torch.empty(m.NG, dtype=torch.float32, device=DEV)
        m.ax_f32(1.3, xd, y32)
        e64, e32 = relerr(host(y), yr), relerr(host(y32).astype(np.float64), yr)
        say(f"  schedule {v}: FP64 {e64:.2e} FP32 {e32:.2e}")
        assert e64 <= 1e-12 and e32 <= 2e-5
    m.close()


@pytest.mark.parametrize("mass", [hb.MASS_GWJ, hb.MASS_INVDEG])
def test_dirichlet_mass_kinds(mass):
    m = hb.Mesh(3, 3, 3, 4, jitter=0.05, seed=2, mass=mass, dirichlet=True)
    ref = oracle.Mesh(3, 3, 3, 4, jitter=0.05, seed=2, mass=mass, dirichlet=True)
    x = inputs.random_vector(m.NG, 9)
    y = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    m.ax(0.9, torch.as_tensor(x, device=DEV), y)
    assert relerr(host(y), ref.ax(x, 0.9)) <= 1e-12


def test_dirichlet_cg_history():
    """The small configuration's box (4^3, N=3, jittered) with the boundary masked:
    100 fixed iterations against the oracle's residual history."""
    c = inputs.PLAIN_SMALL
    say("[case] Dirichlet CG history, 4^3 N=3")
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, dirichlet=True)
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, dirichlet=True)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, c.rhs_seed)
    bh = oracle.rhs(m.NG, c.rhs_seed)
    assert np.array_equal(host(b), bh)
    x = torch.empty_like(b)
    res = m.cg(c.lam, b, x, max_iter=100, fixed_iters=True)
    assert res.status == hb.HB_OK and res.iters == 100
    href, bar = history_bar(ref, bh, c.lam, 100)
    ratio = compare_history(res.history, href, bar)
    say(f"history ratio to bar: {ratio:.3f}")
    assert ratio <= 1.0


@pytest.mark.parametrize("prec", [hb.PREC_FP64, hb.PREC_FP32_RR, hb.PREC_FP32_IR])
def test_dirichlet_tolerance_solves(prec):
    m = hb.Mesh(4, 3, 3, 5, jitter=0.05, seed=3, fp32=True, dirichlet=True)
    ref = oracle.Mesh(4, 3, 3, 5, jitter=0.05, seed=3, dirichlet=True)
    b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
    hb.rhs_uniform(b, 17)
    x = torch.empty_like(b)
    res = m.cg(1.0, b, x, max_iter=20000, fixed_iters=False, rtol=1e-10, prec=prec)
    assert res.status == hb.HB_OK, res
    bh = oracle.rhs(m.NG, 17)
    tr = np.linalg.norm(bh - ref.ax(host(x), 1.0)) / np.linalg.norm(bh)
    say(f"prec {prec}: iters {res.iters} true residual {tr:.2e}")
    assert tr <= 1.2e-10


def test_dirichlet_batch_and_engine():
    cases = [inputs.BoxCase("d0", 3, 3, 3, 3, 0.05, 1, 31), inputs.BoxCase("d1", 2, 3, 2, 7, 0.05, 2, 32),
             inputs.BoxCase("d2", 2, 2, 2, 9, 0.05, 3, 33)]
    ms, bs = [], []
    for c in cases:
        m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=True, dirichlet=True)
        b = torch.empty(m.NG, dtype=torch.float64, device=DEV)
        hb.rhs_uniform(b, c.rhs_seed)
        ms.append(m)
        bs.append(b)
    xs = [torch.empty_like(b) for b in bs]
    st, res = hb.batch_solve(ms, [c.lam for c in cases], bs, xs, max_iter=20000, rtol=1e-9, prec=hb.PREC_FP32_RR)
    assert st == hb.HB_OK, [r.status for r in res]
    eng = hb.Engine(1 << 30, max_slots=2, prec=hb.PREC_FP32_RR, iters_per_step=10)
    tickets = {eng.submit(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, rhs_seed=c.rhs_seed,
                          rtol=1e-9, dirichlet=True): i for i, c in enumerate(cases)}
    got = {}
    for _ in range(100000):
        if len(got) == len(cases):
            break
        eng.step()
        for t, i in tickets.items():
            if i not in got:
                out = eng.poll(t)
                if out is not None:
                    got[i] = out
    eng.close()
    assert len(got) == len(cases)
    for i, c in enumerate(cases):
        ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, dirichlet=True)
        bh = oracle.rhs(ref.NG, c.rhs_seed)
        for name, xv in (("batch", host(xs[i])), ("engine", got[i][1])):
            assert xv.shape == (ref.NG,)
            tr = np.linalg.norm(bh - ref.ax(xv, c.lam)) / np.linalg.norm(bh)
            say(f"{c.name} {name}: true residual {tr:.2e}")
            assert tr <= 1.2e-9
