"""Work, byte and rate formulas used to report results (host-side arithmetic only).

FLOP counts, byte models and rates follow arXiv:2202.12477:
- NekBone FOM FLOPs per CG iteration, eq. (nekbone_flops);
- operator FLOPs and bytes, the Poisson Operator section, and its roofline eq. (op_perf);
- hipBone CG FLOPs and bytes per iteration, the Conjugate gradient Iteration section, eq. (hipbone_flops);
- throughput, eq. (throughput).
The fused-assembly byte counts describe this library's kernels (y is assembled
in place, so the local vector y_L and the CSR gather of the paper's two-phase
operator never reach memory).
"""
from __future__ import annotations

import math


def nekbone_flops(E: int, N: int) -> float:
    """FLOPs per CG iteration counted by NekBone for its figure of merit."""
    return 12.0 * E * (N + 1) ** 4 + 34.0 * E * (N + 1) ** 3


def hipbone_cg_flops(E: int, N: int) -> float:
    """FLOPs per hipBone CG iteration (operator, gather, vector updates)."""
    return 12.0 * E * (N + 1) ** 4 + 19.0 * E * (N + 1) ** 3 + 10.0 * E * N ** 3


def ax_flops(E: int, N: int) -> float:
    """FLOPs of one screened-Poisson operator application: D and D^T, G, lambda term."""
    return 12.0 * E * (N + 1) ** 4 + 18.0 * E * (N + 1) ** 3


def ax_bytes_paper(NG: int, NL: int) -> float:
    """The paper's operator kernel bytes with perfect caching (writes y_L)."""
    return 8.0 * NG + 68.0 * NL


def ax_bytes_fused(NG: int, NL: int, word: int = 8) -> float:
    """Fused gather/operator/scatter-add: read x and write y once (N_G each),
    read the 4-byte map and the 7 geometric values per local node."""
    return 2.0 * word * NG + (4.0 + 7.0 * word) * NL


def ax_bytes_two_phase(NG: int, NL: int) -> float:
    """The two-phase operator: the element kernel (x, map, geometry, y_L written:
    8 N_G + 68 N_L), then the gather (y_L read, 4-byte CSR index per local node,
    4-byte row offsets, y written: 12 N_G + 12 N_L)."""
    return ax_bytes_paper(NG, NL) + 12.0 * NG + 12.0 * NL


def ax_bytes_f32(NG: int, NL: int) -> float:
    """FP32 operator: FP64 x read, FP32 y written, int32 map, 7 FP32 geometric values."""
    return 8.0 * NG + 4.0 * NG + (4.0 + 7.0 * 4.0) * NL


def cg_iter_bytes_paper(NG: int, NL: int) -> float:
    """Bytes per hipBone CG iteration, two-phase operator and separate vector kernels."""
    return 108.0 * NG + 80.0 * NL


def cg_iter_bytes_fused(NG: int, NL: int) -> float:
    """Bytes per CG iteration of this library: the fused operator, one residual
    kernel (r -= alpha Ap, r.r: 24 N_G) and one update kernel (x += alpha p,
    p = r + beta p, Ap = 0 for the next assembly: 48 N_G)."""
    return ax_bytes_fused(NG, NL) + 24.0 * NG + 48.0 * NG


def op_roofline(N: int, B: float, C: float = math.inf) -> float:
    """eq. (op_perf): min(C, (12(N+1)^4 + 18(N+1)^3) / (8N^3 + 68(N+1)^3) * B)."""
    n1 = N + 1
    return min(C, (12.0 * n1 ** 4 + 18.0 * n1 ** 3) / (8.0 * N ** 3 + 68.0 * n1 ** 3) * B)


def throughput(dofs: float, iters: int, ranks: int, seconds: float) -> float:
    """eq. (throughput): DOFs * CG iterations / (ranks * time)."""
    return dofs * iters / (ranks * seconds)


def fom(E: int, N: int, iters: int, seconds: float) -> float:
    """NekBone figure of merit in FLOP/s."""
    return nekbone_flops(E, N) * iters / seconds


def masked_box_elements(dofs: int, N: int) -> int:
    """Elements per edge n of a Dirichlet-masked cube with (nN-1)^3 DOFs."""
    side = round(dofs ** (1.0 / 3.0))
    if side ** 3 != dofs or (side + 1) % N:
        raise ValueError(f"{dofs} is not (nN-1)^3 for N={N}")
    return (side + 1) // N
