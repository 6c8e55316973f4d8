"""Profiling driver for rocprofv3: operator launches plus a streaming kernel of known traffic.

Runs `--launches` applications of the operator (y += A x, hb_ax_add; the FP32
operator with --fp32; the two-phase operator, y = A x on an HB_MESH_GATHER
mesh, with --gather) on one synthetic box, then as many launches of the 8:1
streaming probe (hb_stream_probe over 2^25 outputs: 8 * 2^25 doubles read and
2^25 written per launch, 2.4 GB).  Under `rocprofv3 --pmc FETCH_SIZE` (then
WRITE_SIZE, in a run of its own) the probe's counter values per launch, divided
by its known bytes, give the factor that turns the counters into HBM bytes for
the operator's launches.

  python -m paper_2202_12477_amd.profile_ax [--case box32_N7_affine | sweepN] [--launches K] [--fp32 | --gather]
      [--pcg K] [--cg K]
  python -m paper_2202_12477_amd.profile_ax --cases sweep9 sweep12 sweep2:fp32 ... [--launches K]

--cases runs several operators one after the other in one process (a case with
the suffix ":fp32" is the FP32 operator on that mesh; "@V" after it runs tile
schedule V instead of the class's default, e.g. sweep11@5 or sweep11:fp32@0), so
that one profiler pass covers them all; each case's launches are announced on
stdout first.

--pcg K then also runs K fixed iterations of Jacobi-preconditioned FP64 CG on
the same mesh (its vector kernels: residual_kernel<double, true>,
update_kernel<double, true, ...>); --cg K the same with plain CG
(residual_kernel<double, false>, update_kernel<double, false, ...>).
"""
from __future__ import annotations

import argparse
import os
import sys

STREAM_N = 1 << 25


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", default="box32_N7_affine", help="box32_N7_affine, box4_N3_jitter or sweep<N>")
    ap.add_argument("--dirichlet", action="store_true", help="the case's box with its boundary nodes masked")
    ap.add_argument("--n", type=int, default=0, help="override the case's elements per edge (cubic box)")
    ap.add_argument("--launches", type=int, default=10)
    ap.add_argument("--fp32", action="store_true")
    ap.add_argument("--gather", action="store_true")
    ap.add_argument("--pcg", type=int, default=0)
    ap.add_argument("--cg", type=int, default=0)
    ap.add_argument("--cases", nargs="*", default=None, help="several cases (suffix :fp32 for the FP32 operator)")
    args = ap.parse_args()
    if args.cases:
        return run_cases(args.cases, args.launches)
    if args.fp32 and args.gather:
        ap.error("the two-phase operator is FP64 only")

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import inputs
    import paper_2202_12477_amd as hb

    if args.case.startswith("sweep"):
        c = inputs.order_sweep_case(int(args.case[5:]))
    else:
        c = {k.name: k for k in (inputs.PLAIN_SMALL, inputs.PLAIN_LARGE)}[args.case]
    nx, ny, nz = (args.n, args.n, args.n) if args.n > 0 else (c.nx, c.ny, c.nz)
    m = hb.Mesh(nx, ny, nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=args.fp32, gather=args.gather,
                dirichlet=args.dirichlet)
    b = torch.empty(m.NG, dtype=torch.float64, device="cuda")
    hb.rhs_uniform(b, c.rhs_seed)
    if args.fp32:
        y = torch.zeros(m.NG, dtype=torch.float32, device="cuda")
        for _ in range(args.launches):
            m.ax_f32(c.lam, b, y)
    elif args.gather:
        y = torch.empty_like(b)
        for _ in range(args.launches):
            m.ax(c.lam, b, y)
    else:
        y = torch.zeros_like(b)
        for _ in range(args.launches):
            m.ax_add(c.lam, b, y)
    if args.cg > 0:
        x = torch.empty_like(b)
        r = m.cg(c.lam, b, x, max_iter=args.cg, fixed_iters=True, history=False)
        assert r.iters == args.cg and r.status == hb.HB_OK, r
        del x
    if args.pcg > 0:
        x = torch.empty_like(b)
        r = m.cg(c.lam, b, x, max_iter=args.pcg, fixed_iters=True, history=False, precond=hb.PRECOND_JACOBI)
        assert r.iters == args.pcg and r.status == hb.HB_OK, r
        del x
    torch.cuda.synchronize()
    print(f"operator {c.name}{' dirichlet' if args.dirichlet else ''} E={m.E} N={c.N} NG={m.NG} NL={m.NL} launches={args.launches} pcg={args.pcg} cg={args.cg} "
          f"{'fp32' if args.fp32 else 'fp64'}{' two-phase' if args.gather else ''}", flush=True)
    m.close()
    del b, y
    inp = torch.ones(8 * STREAM_N, dtype=torch.float64, device="cuda")
    out = torch.empty(STREAM_N, dtype=torch.float64, device="cuda")
    for _ in range(args.launches):
        hb.stream_probe(inp, out)
    torch.cuda.synchronize()
    print(f"stream probe n={STREAM_N} read_bytes={8 * 8 * STREAM_N} write_bytes={8 * STREAM_N} "
          f"launches={args.launches}", flush=True)


def run_cases(cases, launches):
    """Operator launches on several order-sweep meshes (or the named boxes), then the probe."""
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import inputs
    import paper_2202_12477_amd as hb

    named = {k.name: k for k in (inputs.PLAIN_SMALL, inputs.PLAIN_LARGE)}
    for spec in cases:
        spec, _, sched = spec.partition("@")
        name, _, kind = spec.partition(":")
        fp32 = kind == "fp32"
        c = inputs.order_sweep_case(int(name[5:])) if name.startswith("sweep") else named[name]
        prec = hb.PREC_FP32_RR if fp32 else hb.PREC_FP64
        saved = hb.get_schedule(c.N, prec)
        if sched:
            hb.set_schedule(c.N, prec, int(sched))
        m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=fp32)
        b = torch.empty(m.NG, dtype=torch.float64, device="cuda")
        hb.rhs_uniform(b, c.rhs_seed)
        print(f"operator {c.name} E={m.E} N={c.N} NG={m.NG} NL={m.NL} launches={launches} "
              f"{'fp32' if fp32 else 'fp64'} schedule={hb.get_schedule(c.N, hb.PREC_FP32_RR if fp32 else hb.PREC_FP64)}",
              flush=True)
        if fp32:
            y = torch.zeros(m.NG, dtype=torch.float32, device="cuda")
            for _ in range(launches):
                m.ax_f32(c.lam, b, y)
        else:
            y = torch.zeros_like(b)
            for _ in range(launches):
                m.ax_add(c.lam, b, y)
        torch.cuda.synchronize()
        m.close()
        del b, y
        if sched:
            hb.set_schedule(c.N, prec, saved)
    inp = torch.ones(8 * STREAM_N, dtype=torch.float64, device="cuda")
    out = torch.empty(STREAM_N, dtype=torch.float64, device="cuda")
    for _ in range(launches):
        hb.stream_probe(inp, out)
    torch.cuda.synchronize()
    print(f"stream probe n={STREAM_N} read_bytes={8 * 8 * STREAM_N} write_bytes={8 * STREAM_N} "
          f"launches={launches}", flush=True)


if __name__ == "__main__":
    main()
