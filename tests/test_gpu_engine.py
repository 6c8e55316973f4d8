"""Continuous-batching engine (hb_engine_*) on the GPU.

Requests arrive while others run, are admitted as slots and budget free up,
share launches with the running ones, and are retired individually.  Each
result must be the same alone and in the mix, within the tolerance it was
solved to: ||A (x_mix - x_alone)|| <= 2 tol ||b||, and each one's true
residual (FP64 oracle operator) meets the tolerance.
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

TOL = 1e-8
REQS = [inputs.BoxCase("r0", 2, 2, 2, 3, 0.05, 1, 101), inputs.BoxCase("r1", 3, 2, 2, 5, 0.05, 2, 102),
        inputs.BoxCase("r2", 1, 1, 1, 11, 0.0, 3, 103), inputs.BoxCase("r3", 4, 4, 3, 3, 0.05, 4, 104),
        inputs.BoxCase("r4", 2, 2, 2, 7, 0.05, 5, 105), inputs.BoxCase("r5", 3, 3, 3, 9, 0.05, 6, 106),
        inputs.BoxCase("r6", 5, 1, 1, 3, 0.0, 7, 107), inputs.BoxCase("r7", 2, 3, 2, 5, 0.05, 8, 108)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def alone(c, prec):
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=prec != hb.PREC_FP64)
    b = torch.empty(m.NG, dtype=torch.float64, device="cuda")
    hb.rhs_uniform(b, c.rhs_seed)
    x = torch.empty_like(b)
    r = m.cg(c.lam, b, x, max_iter=100000, fixed_iters=False, rtol=TOL, prec=prec)
    assert r.status == hb.HB_OK
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.mark.parametrize("prec,graphs", [(hb.PREC_FP64, False), (hb.PREC_FP32_RR, False), (hb.PREC_FP64, True),
                                         (hb.PREC_FP32_RR, True)])
def test_engine_mix_equals_alone(prec, graphs):
    say(f"[case] engine prec={prec} graphs={graphs}")
    # a budget for about three of the larger requests at a time forces queueing
    fps = [hb.request_footprint(c.nx, c.ny, c.nz, c.N, prec, 100000) for c in REQS]
    budget = 3 * max(fps)
    eng = hb.Engine(budget, max_slots=4, prec=prec, max_iter=100000, iters_per_step=20, graphs=graphs)
    tickets = {}
    results = {}
    saw_queue = False
    steps = 0
    # two requests up front, then one more per step (arrivals while others run)
    pending = list(REQS)
    for c in pending[:2]:
        tickets[eng.submit(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, rhs_seed=c.rhs_seed,
                           rtol=TOL)] = c
    pending = pending[2:]
    while len(results) < len(REQS):
        if pending:
            c = pending.pop(0)
            tickets[eng.submit(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, rhs_seed=c.rhs_seed,
                               rtol=TOL)] = c
        info = eng.step()
        steps += 1
        assert info["used_bytes"] <= budget
        assert info["running"] <= 4
        saw_queue = saw_queue or info["queued"] > 0
        for t, c in tickets.items():
            if t in results:
                continue
            out = eng.poll(t)
            if out is not None:
                results[t] = out
        assert steps < 100000
    assert saw_queue, "the budget never made a request wait"
    for t, c in tickets.items():
        r, x = results[t]
        assert r.status == hb.HB_OK, (c.name, r)
        ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
        bh = oracle.rhs(ref.NG, c.rhs_seed)
        tr = np.linalg.norm(bh - ref.ax(x, c.lam)) / np.linalg.norm(bh)
        xa = alone(c, prec)
        d = np.linalg.norm(ref.ax(x - xa, c.lam)) / np.linalg.norm(bh)
        say(f"{c.name}: iters {r.iters} true residual {tr:.2e}, |A(x_mix - x_alone)|/|b| {d:.2e}")
        assert tr <= 1.2 * TOL
        assert d <= 2.2 * TOL
    eng.close()


def test_engine_follows_a_schedule_change_between_steps():
    """Changing a class's tile schedule while requests are admitted: the engine
    rebuilds its work lists (tile counts and order) before the next step."""
    say("[case] engine schedule change between steps")
    cases = [REQS[4], REQS[5], REQS[3]]  # N = 7, 9, 3
    old = {c.N: hb.get_schedule(c.N, hb.PREC_FP64) for c in cases}
    new = {7: 0 if old[7] != 0 else 3, 9: 1 if old[9] != 1 else 0, 3: 2 if old[3] != 2 else 1}
    eng = hb.Engine(8 << 30, max_slots=4, prec=hb.PREC_FP64, max_iter=100000, iters_per_step=5, graphs=True)
    try:
        tickets = {eng.submit(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, rhs_seed=c.rhs_seed,
                              rtol=TOL): c for c in cases}
        eng.step()
        eng.step()
        for N, v in new.items():
            hb.set_schedule(N, hb.PREC_FP64, v)
        results = {}
        for _ in range(100000):
            if len(results) == len(cases):
                break
            eng.step()
            for t in tickets:
                if t not in results:
                    out = eng.poll(t)
                    if out is not None:
                        results[t] = out
        assert len(results) == len(cases)
    finally:
        for N, v in old.items():
            hb.set_schedule(N, hb.PREC_FP64, v)
        eng.close()
    for t, c in tickets.items():
        r, x = results[t]
        assert r.status == hb.HB_OK, (c.name, r)
        ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
        bh = oracle.rhs(ref.NG, c.rhs_seed)
        tr = np.linalg.norm(bh - ref.ax(x, c.lam)) / np.linalg.norm(bh)
        say(f"{c.name}: iters {r.iters} true residual {tr:.2e}")
        assert tr <= 1.2 * TOL


def test_engine_reports_host_time_per_phase():
    """hb_engine_info's cumulative host times: admission, iterations and
    retirement are each counted, grow monotonically, and add up to no more than
    the wall time of the steps."""
    import time

    say("[case] engine phase times")
    eng = hb.Engine(4 << 30, max_slots=2, prec=hb.PREC_FP64, max_iter=100000, iters_per_step=10)
    try:
        tickets = [eng.submit(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, rhs_seed=c.rhs_seed, rtol=TOL)
                   for c in REQS[:3]]
        last = dict(admit_s=0.0, iterate_s=0.0, retire_s=0.0)
        wall, done = 0.0, set()
        for _ in range(100000):
            if len(done) == len(tickets):
                break
            t0 = time.perf_counter()
            info = eng.step()
            wall += time.perf_counter() - t0
            for k in last:
                assert info[k] >= last[k]
                last[k] = info[k]
            for t in tickets:
                if t not in done and eng.poll(t, want_x=False) is not None:
                    done.add(t)
        assert len(done) == len(tickets)
    finally:
        eng.close()
    say(f"  {last}, steps' wall {wall:.3f} s")
    assert last["admit_s"] > 0 and last["iterate_s"] > 0 and last["retire_s"] > 0
    assert sum(last.values()) <= wall + 1e-3


def test_engine_rejects_requests_larger_than_budget():
    eng = hb.Engine(10 << 20, max_slots=2, prec=hb.PREC_FP64)
    with pytest.raises(hb.HbError) as e:
        eng.submit(16, 16, 16, 7)
    assert e.value.status == hb.HB_ERR_BUDGET
    t = eng.submit(2, 2, 2, 3, rhs_seed=5)
    while eng.poll(t, want_x=False) is None:
        eng.step()
    eng.close()


def test_request_loops_replay_a_trace():
    """The request loops behind the serving measurement: both solve every request
    of a timed trace and report consistent latency summaries."""
    from paper_2202_12477_amd import serving

    say("[case] serving request loops on a 4-request trace")
    trace = [(0.0, REQS[0]), (0.001, REQS[1]), (0.002, REQS[6]), (0.05, REQS[3])]
    a = serving.replay_engine(trace, prec=hb.PREC_FP32_RR, hbm_budget=1 << 30, max_slots=2, iters_per_step=10)
    b = serving.replay_sequential(trace)
    say(f"engine {a}\nsequential {b}")
    for r in (a, b):
        assert r["requests"] == 4 and r["solves_per_s"] > 0 and r["cg_iterations"] > 0
        assert 0 < r["p50_s"] <= r["p99_s"] <= r["wall_s"]
    assert a["engine_steps"] >= 1


def test_serving_workload_full_size():
    """The first 48 arrivals of the serving trace at their full sizes (up to 40M
    local nodes per request), through the engine configured as in the serving
    measurement (FP32 operator with FP64 residual replacement, 64 GB budget, 32
    slots, 25 iterations per step, quotas).  Every request must finish with its
    FP64 true residual (computed on the device by the engine) within 1e-8; the
    requests the oracle handles in about a second (up to 5M local nodes) are
    checked again with the oracle's FP64 operator."""
    trace = inputs.serving_trace(48)
    say(f"[case] serving workload, {len(trace)} requests at full size")
    eng = hb.Engine(64 << 30, max_slots=32, prec=hb.PREC_FP32_RR, max_iter=200000, iters_per_step=25)
    try:
        tickets = {eng.submit(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, rhs_seed=c.rhs_seed,
                              lam=c.lam, rtol=TOL): c for _, c in trace}
        results = {}
        steps = 0
        while len(results) < len(tickets):
            eng.step()
            steps += 1
            for t, c in tickets.items():
                if t not in results:
                    out = eng.poll(t)
                    if out is not None:
                        results[t] = out
                        if len(results) % 8 == 0:
                            say(f"{len(results)} done after {steps} steps")
            assert steps < 200000
    finally:
        eng.close()
    checked = 0
    for t, c in tickets.items():
        r, x = results[t]
        assert r.status == hb.HB_OK, (c.name, r)
        assert r.res <= TOL * r.bnorm * 1.0000001, (c.name, r.res / r.bnorm)
        if c.nx * c.ny * c.nz * (c.N + 1) ** 3 <= 5_000_000:
            ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
            bh = oracle.rhs(ref.NG, c.rhs_seed)
            tr = np.linalg.norm(bh - ref.ax(x, c.lam)) / np.linalg.norm(bh)
            assert tr <= 1.2 * TOL, (c.name, tr)
            checked += 1
    say(f"{checked} of {len(tickets)} requests checked against the oracle")
    assert checked >= 40
