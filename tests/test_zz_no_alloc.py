"""hb_cg_solve_noalloc (the solve without device allocation) against hb_cg_solve,
through the C ABI: two calls in a row on one GPU, the second on a smaller
problem (the static workspace keeps the first call's contents), fixed-count and
tolerance solves, with and without the Jacobi preconditioner; both sides held to
the oracle's residual history, and the no-allocation call leaves the mesh's
device footprint unchanged."""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_12477_amd as hb
from cg_envelope import compare_history, history_bar

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def solve_both(nx, ny, nz, N, jitter, seed, rhs_seed, **kw):
    m = hb.Mesh(nx, ny, nz, N, jitter=jitter, seed=seed)
    b = torch.from_numpy(oracle.rhs(m.NG, rhs_seed)).to(DEV)
    before = m.device_bytes()
    x0 = torch.full_like(b, float("nan"))  # x0_zero: the initial content is ignored
    r0 = m.cg_noalloc(1.0, b, x0, **kw)
    assert m.device_bytes() == before, "the no-allocation solve allocated mesh workspace"
    x1 = torch.empty_like(b)
    r1 = m.cg(1.0, b, x1, **kw)
    torch.cuda.synchronize()
    return m, b, (r0, x0.cpu().numpy()), (r1, x1.cpu().numpy())


@pytest.mark.parametrize("precond", [hb.PRECOND_NONE, hb.PRECOND_JACOBI])
def test_two_calls_fixed_count(precond):
    # first call: 6x5x4 elements at N=5 (ragged), then a smaller 3x3x3 box at N=3
    for (nx, ny, nz, N, seed, rs) in [(6, 5, 4, 5, 21, 31), (3, 3, 3, 3, 22, 32)]:
        say(f"[case] noalloc fixed {nx}x{ny}x{nz} N={N} precond={precond}")
        m, b, (ra, xa), (rb, xb) = solve_both(nx, ny, nz, N, 0.05, seed, rs, max_iter=60, fixed_iters=True,
                                              precond=precond)
        assert ra.status == rb.status == hb.HB_OK
        assert ra.iters == rb.iters == 60
        ref = oracle.Mesh(nx, ny, nz, N, jitter=0.05, seed=seed)
        bh = b.cpu().numpy()
        if precond == hb.PRECOND_NONE:
            href, bar = history_bar(ref, bh, 1.0, 60)
            assert compare_history(ra.history, href, bar) <= 1.0
            assert compare_history(rb.history, href, bar) <= 1.0
        # the two entry points run the same kernels: equal up to the order of atomic additions
        h_a, h_b = np.array(ra.history), np.array(rb.history)
        live = h_b / h_b[0] > 1e-13
        assert np.max(np.abs(h_a - h_b)[live] / h_b[live]) <= 1e-10
        assert relerr(xa, xb) <= 1e-9
        assert ra.res0 == pytest.approx(rb.res0, rel=1e-14)
        assert ra.bnorm == pytest.approx(rb.bnorm, rel=1e-14)
        m.close()


def test_two_calls_tolerance():
    for (nx, ny, nz, N, seed, rs) in [(5, 4, 4, 4, 23, 33), (2, 3, 2, 6, 24, 34)]:
        say(f"[case] noalloc tolerance {nx}x{ny}x{nz} N={N}")
        m, b, (ra, xa), (rb, xb) = solve_both(nx, ny, nz, N, 0.05, seed, rs, max_iter=3000, fixed_iters=False,
                                              rtol=1e-9, check_every=10)
        assert ra.status == rb.status == hb.HB_OK
        assert abs(ra.iters - rb.iters) <= 1
        ref = oracle.Mesh(nx, ny, nz, N, jitter=0.05, seed=seed)
        bh = b.cpu().numpy()
        out = ref.cg(bh, 1.0, max_iter=3000, rtol=1e-9)
        assert abs(ra.iters - out["iters"]) <= 1
        # the true residual of the no-allocation solution, from the oracle's operator
        assert np.linalg.norm(bh - ref.ax(xa, 1.0)) <= 2e-9 * np.linalg.norm(bh)
        assert relerr(xa, xb) <= 1e-7
        m.close()


def test_rejects_what_does_not_fit():
    say("[case] noalloc rejections")
    m = hb.Mesh(24, 24, 24, 7)  # 4.9M DOFs: more than the 64 MiB buffer holds
    b = torch.zeros(m.NG, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    with pytest.raises(hb.HbError) as ei:
        m.cg_noalloc(1.0, b, x, max_iter=10)
    assert ei.value.status == hb.HB_ERR_INVALID_ARG and "no-allocation buffer" in str(ei.value)
    m.close()
    small = hb.Mesh(2, 2, 2, 3)
    b = torch.zeros(small.NG, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    with pytest.raises(hb.HbError) as ei:  # an iteration cap whose histories overflow the buffer
        small.cg_noalloc(1.0, b, x, max_iter=5_000_000)
    assert ei.value.status == hb.HB_ERR_INVALID_ARG
    small.close()
