"""Request loops over a timed arrival trace: the continuous-batching engine and
the plain one-at-a-time FP64 solver, with per-request latency.

A trace is a list of (arrival_seconds, request) where a request has the fields
nx, ny, nz, N, jitter, mesh_seed, rhs_seed and lam (for example
`inputs.serving_trace`).  Time starts when the loop starts; a request's
latency is its completion time minus its arrival time, so it includes queueing.
Both loops solve every request to the same relative residual and fail loudly on
any request that does not reach it.  Progress lines (every `progress` completed
requests) go to stderr.
"""
from __future__ import annotations

import sys
import time

import numpy as np

from . import HB_OK, PREC_FP64, Engine, Mesh, rhs_uniform


def _summary(lat, wall, iters, extra=None):
    lat = np.asarray(lat)
    out = {"requests": int(lat.size), "wall_s": round(wall, 3), "solves_per_s": round(lat.size / wall, 3),
           "p50_s": round(float(np.percentile(lat, 50)), 4) if lat.size else None,
           "p99_s": round(float(np.percentile(lat, 99)), 4) if lat.size else None,
           "mean_s": round(float(lat.mean()), 4) if lat.size else None, "cg_iterations": int(iters)}
    if extra:
        out.update(extra)
    return out


def _budget_extra(trace, budget, wall, done):
    """Counts of a run cut off after `budget` seconds (it ended at `wall`): requests
    that had arrived by the cut-off, completed, and left unfinished (queued or
    running), and the completion rate over the budget."""
    offered = sum(1 for arrival, _ in trace if arrival <= min(budget, wall))
    return {"budget_s": budget, "offered": offered, "completed": done, "backlog": offered - done,
            "completed_per_s": round(done / budget, 3)}


def replay_engine(trace, *, prec, rtol=1e-8, hbm_budget=64 << 30, max_slots=32, iters_per_step=25,
                  max_iter=200000, precond=0, progress=None, budget=None, autotune=False):
    """Submit each request when its arrival time has passed, step the engine while
    anything is queued or running, and poll for completions after every step.
    With `budget` (seconds) the loop stops at that wall time: the summary covers the
    requests completed by then and counts those offered and left unfinished."""
    import torch

    eng = Engine(hbm_budget, max_slots=max_slots, prec=prec, max_iter=max_iter, iters_per_step=iters_per_step,
                 precond=precond, autotune=autotune)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nxt, lat, iters, steps, waiting = 0, [], 0, 0, {}
        info = {}
        while len(lat) < len(trace):
            now = time.perf_counter() - t0
            if budget is not None and now >= budget:
                break
            while nxt < len(trace) and trace[nxt][0] <= now:
                arrival, c = trace[nxt]
                t = eng.submit(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, rhs_seed=c.rhs_seed,
                               lam=c.lam, rtol=rtol)
                waiting[t] = arrival
                nxt += 1
            if not waiting:
                pause = trace[nxt][0] - (time.perf_counter() - t0)
                if budget is not None:
                    pause = min(pause, budget - (time.perf_counter() - t0))
                time.sleep(max(0.0, pause))
                continue
            info = eng.step()
            ready = info["completed"]  # results waiting to be polled
            steps += 1
            for t in list(waiting):
                if ready == 0:
                    break
                got = eng.poll(t, want_x=False)
                if got is None:
                    continue
                ready -= 1
                res = got[0]
                if res.status != HB_OK:
                    raise RuntimeError(f"request {t} ended with status {res.status}")
                lat.append(time.perf_counter() - t0 - waiting.pop(t))
                iters += res.iters
                if progress and len(lat) % progress == 0:
                    print(f"  engine: {len(lat)}/{len(trace)} done at {time.perf_counter() - t0:.1f} s",
                          file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
    finally:
        eng.close()
    # host wall time the engine spent per phase of its steps (admission and
    # retirement leave the device without engine work)
    extra = {"engine_steps": steps, **{k: round(info.get(k, 0.0), 3) for k in ("admit_s", "iterate_s", "retire_s")}}
    if budget is not None:
        extra.update(_budget_extra(trace, budget, wall, len(lat)))
    return _summary(lat, wall, iters, extra)


def replay_sequential(trace, *, rtol=1e-8, max_iter=200000, progress=None, budget=None):
    """One request at a time in arrival order, FP64 CG (hb_cg_solve), the solution
    copied to the host like the engine's retirement does.  With `budget` (seconds)
    no request starts after that wall time (the one running then completes)."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, iters = [], 0
    for arrival, c in trace:
        now = time.perf_counter() - t0
        if budget is not None and (now >= budget or arrival >= budget):
            break
        if now < arrival:
            time.sleep(arrival - now)
        m = Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
        try:
            b = torch.empty(m.NG, dtype=torch.float64, device="cuda")
            rhs_uniform(b, c.rhs_seed)
            x = torch.empty_like(b)
            res = m.cg(c.lam, b, x, max_iter=max_iter, fixed_iters=False, rtol=rtol, prec=PREC_FP64, history=False)
            x.cpu()
        finally:
            m.close()
        if res.status != HB_OK:
            raise RuntimeError(f"sequential request ended with status {res.status}")
        lat.append(time.perf_counter() - t0 - arrival)
        iters += res.iters
        if progress and len(lat) % progress == 0:
            print(f"  sequential: {len(lat)}/{len(trace)} done at {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    extra = None
    if budget is not None:
        extra = _budget_extra(trace, budget, wall, len(lat))
    return _summary(lat, wall, iters, extra)
