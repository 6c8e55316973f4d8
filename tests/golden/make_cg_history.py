"""Write the oracle's CG residual history of the 32^3 N=7 benchmark configuration.

Calls only ``oracle/``: the 32^3 affine box at N=7 (11,390,625 DOFs), lambda = 1,
U[-1,1) forcing of seed 3, 100 fixed iterations of Algorithm 1, once with
compensated and once with plain left-to-right dot products.  The stored file
holds, per iteration j, ||r_j|| of the compensated run and the per-iteration
bar of the history comparison (1e-10, widened to 10x the spread of the two
summation orders where that exceeds 1e-11).  The two runs go in two threads:
the oracle's C code releases the GIL.

  python tests/golden/make_cg_history.py   # writes tests/golden/cg_history_box32_N7.txt
"""
import os
import sys
import threading
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "cg_history_box32_N7.txt")


def main():
    c = inputs.PLAIN_LARGE
    t0 = time.time()
    m = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    b = oracle.rhs(m.NG, c.rhs_seed)
    print(f"mesh {m.NG} DOFs in {time.time() - t0:.1f} s", flush=True)
    runs = {}

    def run(comp):
        runs[comp] = m.cg(b, c.lam, fixed_iters=c.iters, compensated=comp)["res"]

    th = [threading.Thread(target=run, args=(comp,)) for comp in (True, False)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    ref, alt = runs[True], runs[False]
    spread = np.abs(ref - alt) / np.abs(ref)
    bar = np.maximum(1e-10, 10.0 * spread)
    with open(OUT, "w") as f:
        f.write("# Oracle CG residual history of the 32^3 affine box at N=7 (11,390,625 DOFs), lambda=1,\n"
                "# U[-1,1) forcing of seed 3, 100 fixed iterations of Algorithm 1 from x0 = 0.\n"
                "# Written by tests/golden/make_cg_history.py from oracle/ only (plain C, FP64, no FMA).\n"
                "# Columns: j  ||r_j|| (compensated dots)  ||r_j|| (plain dots)  bar_j\n")
        for j in range(len(ref)):
            f.write(f"{j} {ref[j]:.17e} {alt[j]:.17e} {bar[j]:.6e}\n")
    print(f"wrote {OUT} in {time.time() - t0:.1f} s; max spread {spread.max():.3e}", flush=True)


if __name__ == "__main__":
    main()
