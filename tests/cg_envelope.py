"""Per-iteration tolerance for comparing CG residual histories with the oracle.

The bar is 1e-10 relative.  Unpreconditioned CG amplifies rounding in its
late iterations, so two correct FP64 runs that differ only in summation order
drift apart there; where the oracle's own two orders (compensated and plain
dot products) differ by more than 1e-11, the bar at that iteration is 10x
their spread.  Iterations whose reference residual is below 1e-13 of the first
are at the rounding floor and are not compared.
"""
import numpy as np


def history_bar(mesh, b, lam, iters):
    """Return (reference residual history, per-iteration relative bar)."""
    ref = mesh.cg(b, lam, fixed_iters=iters, compensated=True)["res"]
    alt = mesh.cg(b, lam, fixed_iters=iters, compensated=False)["res"]
    spread = np.abs(ref - alt) / np.abs(ref)
    return ref, np.maximum(1e-10, 10.0 * spread)


def compare_history(got, ref, bar):
    """Max ratio |got-ref|/(|ref| bar) over the iterations above the rounding floor (<= 1 passes)."""
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    live = ref / ref[0] > 1e-13
    return float(np.max(np.abs(got - ref)[live] / (np.abs(ref[live]) * bar[live])))
