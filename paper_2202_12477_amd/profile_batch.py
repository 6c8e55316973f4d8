"""Profiling driver for rocprofv3: the batched and the served workloads.

  python -m paper_2202_12477_amd.profile_batch --case batch [--prec fp32rr|fp64] [--graph-k K] [--jacobi]
      the 64 uneven problems of the batched workload, one hb_batch_solve to 1e-8
  python -m paper_2202_12477_amd.profile_batch --case serve [--requests R] [--prec fp32rr|fp64] [--jacobi]
      the first R arrivals of the serving trace through the engine (64 GB budget,
      32 slots, 25 iterations per step)

--jacobi solves with the Jacobi preconditioner.

Prints one summary line per run (solves/s, iterations), nothing else.
"""
from __future__ import annotations

import argparse
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=("batch", "serve"), default="batch")
    ap.add_argument("--prec", choices=("fp32rr", "fp64"), default="fp32rr")
    ap.add_argument("--graph-k", type=int, default=0)
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--jacobi", action="store_true")
    args = ap.parse_args()

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import inputs
    import paper_2202_12477_amd as hb

    prec = hb.PREC_FP32_RR if args.prec == "fp32rr" else hb.PREC_FP64
    precond = hb.PRECOND_JACOBI if args.jacobi else hb.PRECOND_NONE
    tag = f"{args.prec}{' jacobi' if args.jacobi else ''}"
    if args.case == "batch":
        cases = inputs.batched_cases()
        ms, bs = [], []
        for c in cases:
            m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=prec != hb.PREC_FP64)
            b = torch.empty(m.NG, dtype=torch.float64, device="cuda")
            hb.rhs_uniform(b, c.rhs_seed)
            ms.append(m)
            bs.append(b)
        xs = [torch.empty_like(b) for b in bs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, res = hb.batch_solve(ms, [c.lam for c in cases], bs, xs, max_iter=100000, rtol=1e-8, prec=prec,
                                 graph_k=args.graph_k, precond=precond)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert st == hb.HB_OK, [r.status for r in res]
        print(f"batch {len(cases)} problems {tag} graph_k={args.graph_k}: {len(cases) / dt:.2f} solves/s, "
              f"{sum(r.iters for r in res)} iterations", flush=True)
        for m in ms:
            m.close()
    else:
        from paper_2202_12477_amd import serving

        out = serving.replay_engine(inputs.serving_trace(args.requests), prec=prec, precond=precond)
        print(f"serve {args.requests} requests {tag}: {out}", flush=True)


if __name__ == "__main__":
    main()
