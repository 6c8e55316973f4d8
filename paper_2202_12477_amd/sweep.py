"""Per-degree measurements on the order-sweep meshes (about 2^24 local nodes each).

For every degree N: the FP64 operator (hb_ax_add) and the FP32 operator
(hb_ax_f32: output cleared, then the operator) timed with HIP events on the
launching stream (median of three runs after 128 untimed launches), as
algorithmic GB/s and GDOF/s; the FP32 operator's relative
difference from the FP64 one on the same input; and with --solve, FP64 CG vs
the two mixed-precision solvers to a relative residual (solves timed end to
end, true residual reported by each solver); with --two-phase, y = A x by the
two-phase operator (HB_MESH_GATHER: element kernel, then the gather) beside
the fused hb_ax on the same mesh, in the paper's operator GFLOP/s.  One JSON
line per degree.

  python -m paper_2202_12477_amd.sweep [--degrees 1 2 ...] [--reps 20] [--solve] [--rtol 1e-10] [--two-phase]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--degrees", type=int, nargs="*", default=list(range(1, 16)))
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--solve", action="store_true")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--two-phase", action="store_true")
    args = ap.parse_args()

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import inputs
    import paper_2202_12477_amd as hb
    from paper_2202_12477_amd import metrics

    def timed(fn, reps):
        # 128 untimed launches (after each mesh's host set-up the device has been
        # idle, and its first ~100 launches run up to 15% slow at FP64 N = 9-12),
        # then the median of three timed runs of `reps` launches
        for _ in range(128):
            fn()
        torch.cuda.synchronize()
        runs = []
        for _ in range(3):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(reps):
                fn()
            e.record()
            e.synchronize()
            runs.append(s.elapsed_time(e) * 1e-3 / reps)
        return sorted(runs)[1]

    for N in args.degrees:
        c = inputs.order_sweep_case(N)
        m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=True)
        b = torch.empty(m.NG, dtype=torch.float64, device="cuda")
        hb.rhs_uniform(b, c.rhs_seed)
        y = torch.zeros_like(b)
        y32 = torch.zeros(m.NG, dtype=torch.float32, device="cuda")
        t64 = timed(lambda: m.ax_add(c.lam, b, y), args.reps)
        t32 = timed(lambda: m.ax_f32(c.lam, b, y32), args.reps)
        m.ax(c.lam, b, y)
        m.ax_f32(c.lam, b, y32)
        diff = float(torch.linalg.norm(y32.double() - y) / torch.linalg.norm(y))
        # hb_ax_f32 clears its output first (4 N_G bytes) and then runs the FP32 operator
        b64, b32 = metrics.ax_bytes_fused(m.NG, m.NL), metrics.ax_bytes_f32(m.NG, m.NL) + 4.0 * m.NG
        out = {"N": N, "n": c.nx, "E": m.E, "n_local": m.NL, "n_global": m.NG,
               "fp64_us": round(t64 * 1e6, 1), "fp64_GBs": round(b64 / t64 / 1e9, 1),
               "fp64_gdofs": round(m.NG / t64 / 1e9, 2), "fp64_gflops": round(metrics.ax_flops(m.E, N) / t64 / 1e9, 1),
               "fp32_us": round(t32 * 1e6, 1), "fp32_GBs": round(b32 / t32 / 1e9, 1),
               "fp32_gdofs": round(m.NG / t32 / 1e9, 2), "fp32_vs_fp64_rel": float(f"{diff:.3e}")}
        if args.two_phase:
            g = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, gather=True)
            yg = torch.empty_like(b)
            tf = timed(lambda: m.ax(c.lam, b, y), args.reps)
            tg = timed(lambda: g.ax(c.lam, b, yg), args.reps)
            g.ax(c.lam, b, yg)
            m.ax(c.lam, b, y)
            fl = metrics.ax_flops(m.E, N)
            out["two_phase"] = {"fused_ax_us": round(tf * 1e6, 1), "fused_gflops": round(fl / tf / 1e9, 1),
                                "two_phase_us": round(tg * 1e6, 1), "two_phase_gflops": round(fl / tg / 1e9, 1),
                                "two_phase_GBs": round(metrics.ax_bytes_two_phase(m.NG, m.NL) / tg / 1e9, 1),
                                "rel_diff": float(f"{float(torch.linalg.norm(yg - y) / torch.linalg.norm(y)):.3e}")}
            g.close()
            del yg
        if args.solve:
            x = torch.empty_like(b)
            for name, prec in (("fp64", hb.PREC_FP64), ("fp32_ir", hb.PREC_FP32_IR), ("fp32_rr", hb.PREC_FP32_RR)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = m.cg(c.lam, b, x, max_iter=200000, fixed_iters=False, rtol=args.rtol, prec=prec, history=False)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                res = r.res / r.bnorm
                out[f"solve_{name}"] = {"s": round(dt, 4), "iters": r.iters, "outer": r.outer_iters,
                                        "fp64_iters": r.fp64_iters, "status": r.status, "rel_res": float(f"{res:.3e}")}
        print(json.dumps(out), flush=True)
        m.close()
        del b, y, y32


if __name__ == "__main__":
    main()
