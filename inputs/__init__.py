"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds the workload recipes (box sizes, degrees, jitter, seeds) and
a host-side random-vector generator.  It contains none of the method's
arithmetic: the oracle and the GPU library each build the mesh, geometry,
forcing vector and operator themselves from these descriptors.

The paper's workloads are a regular box of hexahedra with a pseudo-random
forcing vector (NekBone and HipBone sections); no public dataset is involved.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class BoxCase:
    """A box mesh of nx*ny*nz hexahedra of degree N on [0,1]^3, unmasked.

    jitter: interior vertices move by up to +-jitter*h per coordinate (0 = affine).
    mesh_seed / rhs_seed: splitmix64 seeds of the vertex jitter and the forcing.
    """

    name: str
    nx: int
    ny: int
    nz: int
    N: int
    jitter: float
    mesh_seed: int
    rhs_seed: int
    lam: float = 1.0
    iters: int = 100

    @property
    def E(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def NL(self) -> int:
        return self.E * (self.N + 1) ** 3

    @property
    def NG(self) -> int:
        return (self.nx * self.N + 1) * (self.ny * self.N + 1) * (self.nz * self.N + 1)

    def with_(self, **kw) -> "BoxCase":
        return replace(self, **kw)


# Plain FP64: 4^3 jittered elements at N=3, 13^3 DOFs, one Ax + 100 CG iterations.
PLAIN_SMALL = BoxCase("box4_N3_jitter", 4, 4, 4, 3, 0.05, 1, 2)
# Plain FP64 at one-GPU scale: 32^3 affine elements at N=7, 225^3 = 11,390,625 DOFs.
PLAIN_LARGE = BoxCase("box32_N7_affine", 32, 32, 32, 7, 0.0, 0, 3)


def order_sweep_case(N: int) -> BoxCase:
    """Order sweep: about 2^24 local nodes at degree N, jittered trilinear mesh."""
    n = int(round((2 ** 24 / (N + 1) ** 3) ** (1.0 / 3.0)))
    return BoxCase(f"sweep_N{N}_n{n}", n, n, n, N, 0.05, 10 + N, 100 + N)


ORDER_SWEEP = [order_sweep_case(N) for N in range(1, 16)]


def random_vector(n: int, seed: int) -> np.ndarray:
    """Standard-normal FP64 vector from numpy's PCG64 stream `seed` (host memory)."""
    return np.random.default_rng(seed).standard_normal(n)


def batched_cases(count: int = 64, master_seed: int = 4) -> list:
    """Uneven independent problems: cubic grids n ~ U{2..24}, N ~ U{3,5,7,9}, each with
    its own jitter seed and forcing seed, lambda = 1 (drawn from numpy's PCG64 stream)."""
    rng = np.random.default_rng(master_seed)
    ns = rng.integers(2, 25, size=count)
    Ns = rng.choice([3, 5, 7, 9], size=count)
    return [BoxCase(f"batch{master_seed}_{i}_n{int(n)}_N{int(N)}", int(n), int(n), int(n), int(N), 0.05,
                    1000 * master_seed + i, 2000 * master_seed + i) for i, (n, N) in enumerate(zip(ns, Ns))]


def serving_window(duration: float, rate: float, master_seed: int = 5) -> list:
    """The arrivals of the serving recipe (serving_trace's request mix, its master
    seed) within the first `duration` seconds at `rate` requests per second."""
    count = int(rate * duration * 2 + 64)
    return [(t, c) for t, c in serving_trace(count, rate, master_seed) if t <= duration]


def serving_trace(count: int, rate: float = 200.0, master_seed: int = 5) -> list:
    """Request stream: Poisson arrivals at `rate` per second; each request is a
    near-cubic box whose element count E* is log-uniform in [8, 32768]
    (nz = floor(E*^(1/3)), ny = floor(sqrt(E*/nz)), nx = round(E*/(ny nz))),
    degree N ~ U{3,5,7,9,11}, jittered, its own seeds, lambda = 1.
    Returns [(arrival_seconds, BoxCase)] for the first `count` arrivals."""
    rng = np.random.default_rng(master_seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    estar = np.exp(rng.uniform(np.log(8.0), np.log(32768.0), size=count))
    Ns = rng.choice([3, 5, 7, 9, 11], size=count)
    out, t = [], 0.0
    for i in range(count):
        t += float(gaps[i])
        e = float(estar[i])
        nz = max(1, int(np.floor(e ** (1.0 / 3.0))))
        ny = max(1, int(np.floor(np.sqrt(e / nz))))
        nx = max(1, int(round(e / (ny * nz))))
        out.append((t, BoxCase(f"req{i}", nx, ny, nz, int(Ns[i]), 0.05, 50000 + i, 60000 + i)))
    return out
