"""Plain FP64 CPU oracle for the assembled SEM screened-Poisson operator and CG.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  The product library
(``paper_2202_12477_amd``) never imports it and it never imports the product:
the two share no code.  ``oracle.c`` holds the arithmetic (see its header for
the citations into arXiv:2202.12477); this module only compiles it with gcc and
marshals numpy arrays through ctypes.  ``brute.py`` is a second, independent
route (dense matrices from numpy's Legendre module and Kronecker products) used
to pin the C oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# No FMA contraction: the oracle computes exactly the operations it spells out.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.{os.getpid()}.tmp"  # per process: parallel test workers build at once
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


# The CPU baseline's timing build: the same source, optimised for the host it
# runs on and multi-threaded with OpenMP (still no FMA contraction).  Built on
# the machine that times it (-march=native), never used by the parity tests.
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
TIMING_CFLAGS = ["-O3", "-march=native", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                 "-std=c11", "-D_GNU_SOURCE"]


def build_timing() -> str:
    """Compile oracle.c into liboracle_omp.so (timing build) with gcc."""
    tmp = f"{_LIB_OMP}.{os.getpid()}.tmp"
    subprocess.check_call(["gcc", *TIMING_CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_OMP)
    return _LIB_OMP


_lib = None
_lib_omp = None


def _declare(L: ctypes.CDLL) -> ctypes.CDLL:
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_int64)
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.oracle_ax_classes.argtypes = [i64, i32, dp, dp, lp, i64, f64, dp, dp, lp, lp, i32]
    L.oracle_ax_classes.restype = None
    L.oracle_cg_classes.argtypes = [i64, i32, dp, dp, lp, i64, f64, dp, dp, i32, i32, f64, i32, dp,
                                    ctypes.POINTER(ctypes.c_int), lp, lp, i32]
    L.oracle_set_threads.argtypes = [i32]
    L.oracle_set_threads.restype = i32
    return L


def timing_lib(build: bool = True) -> ctypes.CDLL:
    """The timing build (compiled here first unless build=False and it exists)."""
    global _lib_omp
    if _lib_omp is None:
        if build or not os.path.exists(_LIB_OMP):
            build_timing()
        _lib_omp = _declare(ctypes.CDLL(_LIB_OMP))
    return _lib_omp


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        i64, i32, u64, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        L.oracle_splitmix64.argtypes = [u64, u64]
        L.oracle_splitmix64.restype = u64
        L.oracle_uniform.argtypes = [u64, u64, u64]
        L.oracle_uniform.restype = f64
        L.oracle_rhs.argtypes = [i64, u64, dp]
        L.oracle_gll.argtypes = [i32, dp, dp]
        L.oracle_deriv.argtypes = [i32, dp, dp]
        L.oracle_vertices.argtypes = [i32, i32, i32, f64, u64, dp]
        L.oracle_map.argtypes = [i32, i32, i32, i32, lp]
        L.oracle_map_dirichlet.argtypes = [i32, i32, i32, i32, lp]
        L.oracle_geometry.argtypes = [i32, i32, i32, i32, dp, i32, dp]
        L.oracle_ax.argtypes = [i64, i32, dp, dp, lp, i64, f64, dp, dp]
        L.oracle_ax.restype = None
        L.oracle_diag.argtypes = [i64, i32, dp, dp, lp, i64, f64, dp]
        L.oracle_diag.restype = None
        L.oracle_pcg.argtypes = [i64, i32, dp, dp, lp, i64, f64, dp, dp, dp, i32, i32, f64, i32, dp,
                                 ctypes.POINTER(ctypes.c_int)]
        L.oracle_cg.argtypes = [i64, i32, dp, dp, lp, i64, f64, dp, dp, i32, i32, f64, i32, dp, dp, dp, dp,
                                ctypes.POINTER(ctypes.c_int)]
        _declare(L)
        _lib = L
    return _lib


def _p(a: np.ndarray, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def splitmix64(state: int, i: int) -> int:
    return int(lib().oracle_splitmix64(state, i))


def uniform(seed: int, stream: int, index: int) -> float:
    return float(lib().oracle_uniform(seed, stream, index))


def rhs(n: int, seed: int) -> np.ndarray:
    b = np.empty(n)
    lib().oracle_rhs(n, seed, _p(b))
    return b


def gll(N: int):
    xi, w = np.empty(N + 1), np.empty(N + 1)
    if lib().oracle_gll(N, _p(xi), _p(w)) != 0:
        raise ValueError("N must be >= 1")
    return xi, w


def deriv(N: int) -> np.ndarray:
    xi, _ = gll(N)
    D = np.empty((N + 1, N + 1))
    lib().oracle_deriv(N, _p(xi), _p(D))
    return D


def vertices(nx: int, ny: int, nz: int, jitter: float, seed: int) -> np.ndarray:
    V = np.empty(((nx + 1) * (ny + 1) * (nz + 1), 3))
    if lib().oracle_vertices(nx, ny, nz, jitter, seed, _p(V)) != 0:
        raise ValueError("bad box")
    return V


MASS_GWJ = 0     # A = S + lambda M   (c = GLL weight x Jacobian)
MASS_INVDEG = 1  # A = S + lambda I   (c = inverse multiplicity W)


@dataclass
class Mesh:
    """Box mesh of nx*ny*nz hexahedra of degree N on [0,1]^3: no masking, or with
    dirichlet=True homogeneous Dirichlet conditions on the boundary of the box (the
    boundary nodes carry no DOF; N_G = (nx N - 1)(ny N - 1)(nz N - 1))."""

    nx: int
    ny: int
    nz: int
    N: int
    jitter: float = 0.0
    seed: int = 0
    mass: int = MASS_GWJ
    dirichlet: bool = False

    def __post_init__(self):
        L = lib()
        n1 = self.N + 1
        self.E = self.nx * self.ny * self.nz
        self.Np = n1 ** 3
        self.NL = self.E * self.Np
        k = -1 if self.dirichlet else 1
        self.NG = (self.nx * self.N + k) * (self.ny * self.N + k) * (self.nz * self.N + k)
        self.xi, self.w = gll(self.N)
        self.D = deriv(self.N)
        self.V = vertices(self.nx, self.ny, self.nz, self.jitter, self.seed)
        self.map = np.empty(self.NL, dtype=np.int64)
        (L.oracle_map_dirichlet if self.dirichlet else L.oracle_map)(self.nx, self.ny, self.nz, self.N,
                                                                      _p(self.map, ctypes.c_int64))
        self.geo = np.empty(self.E * 7 * self.Np)
        st = L.oracle_geometry(self.nx, self.ny, self.nz, self.N, _p(self.V), self.mass, _p(self.geo))
        if st != 0:
            raise ValueError(f"oracle_geometry failed ({st}): non-positive Jacobian?")

    def ax(self, x: np.ndarray, lam: float) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.NG,)
        y = np.empty(self.NG)
        lib().oracle_ax(self.E, self.N, _p(self.D), _p(self.geo), _p(self.map, ctypes.c_int64), self.NG, lam,
                        _p(x), _p(y))
        return y

    def cg(self, b: np.ndarray, lam: float, x0: np.ndarray | None = None, *, fixed_iters: int = 0,
           max_iter: int = 1000, rtol: float = 1e-8, compensated: bool = True):
        """Algorithm 1.  Returns dict(x, iters, status, res, alpha, beta, pap)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.NG) if x0 is None else np.array(x0, dtype=np.float64)
        n = max(fixed_iters, max_iter) + 1
        res, al, be, pap = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
        it = ctypes.c_int(0)
        st = lib().oracle_cg(self.E, self.N, _p(self.D), _p(self.geo), _p(self.map, ctypes.c_int64), self.NG, lam,
                             _p(b), _p(x), max_iter, fixed_iters, rtol, int(compensated), _p(res), _p(al), _p(be),
                             _p(pap), ctypes.byref(it))
        j = it.value
        return dict(x=x, iters=j, status=st, res=res[: j + 1], alpha=al[:j], beta=be[:j], pap=pap[:j])

    def diag(self, lam: float) -> np.ndarray:
        """Diagonal of the assembled operator (the Jacobi preconditioner's M)."""
        d = np.empty(self.NG)
        lib().oracle_diag(self.E, self.N, _p(self.D), _p(self.geo), _p(self.map, ctypes.c_int64), self.NG, lam,
                          _p(d))
        return d

    def pcg(self, b: np.ndarray, lam: float, x0: np.ndarray | None = None, *, fixed_iters: int = 0,
            max_iter: int = 1000, rtol: float = 1e-8, compensated: bool = True, inv: np.ndarray | None = None):
        """Algorithm 1 with the Jacobi preconditioner (inv: M^{-1} as a vector, default
        1/diag(A)).  Returns dict(x, iters, status, res)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.NG) if x0 is None else np.array(x0, dtype=np.float64)
        inv = 1.0 / self.diag(lam) if inv is None else np.ascontiguousarray(inv, dtype=np.float64)
        res = np.zeros(max(fixed_iters, max_iter) + 1)
        it = ctypes.c_int(0)
        st = lib().oracle_pcg(self.E, self.N, _p(self.D), _p(self.geo), _p(self.map, ctypes.c_int64), self.NG, lam,
                              _p(inv), _p(b), _p(x), max_iter, fixed_iters, rtol, int(compensated), _p(res),
                              ctypes.byref(it))
        j = it.value
        return dict(x=x, iters=j, status=st, res=res[: j + 1])

    def classes(self):
        """The 8 element classes of the box, (ex mod 2, ey mod 2, ez mod 2): elements of
        one class share no node.  Returns (order, offsets) as int64 arrays."""
        e = np.arange(self.E, dtype=np.int64)
        ex, ey, ez = e % self.nx, (e // self.nx) % self.ny, e // (self.nx * self.ny)
        key = (ex % 2) + 2 * (ey % 2) + 4 * (ez % 2)
        order = np.argsort(key, kind="stable").astype(np.int64)
        offsets = np.searchsorted(key[order], np.arange(9)).astype(np.int64)
        return order, offsets

    def ax_classes(self, x: np.ndarray, lam: float, L: ctypes.CDLL | None = None) -> np.ndarray:
        """y = A x with the elements swept class by class (on the timing build's
        threads when L is the timing library)."""
        L = L or lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.NG)
        order, offsets = self.classes()
        L.oracle_ax_classes(self.E, self.N, _p(self.D), _p(self.geo), _p(self.map, ctypes.c_int64), self.NG, lam,
                            _p(x), _p(y), _p(order, ctypes.c_int64), _p(offsets, ctypes.c_int64), 8)
        return y

    def cg_classes(self, b: np.ndarray, lam: float, *, fixed_iters: int = 0, max_iter: int = 1000,
                   rtol: float = 1e-8, compensated: bool = True, L: ctypes.CDLL | None = None):
        """Algorithm 1 from x0 = 0 with the class-by-class operator.  Returns dict(x, iters, status, res)."""
        L = L or lib()
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.NG)
        res = np.zeros(max(fixed_iters, max_iter) + 1)
        it = ctypes.c_int(0)
        order, offsets = self.classes()
        st = L.oracle_cg_classes(self.E, self.N, _p(self.D), _p(self.geo), _p(self.map, ctypes.c_int64), self.NG,
                                 lam, _p(b), _p(x), max_iter, fixed_iters, rtol, int(compensated), _p(res),
                                 ctypes.byref(it), _p(order, ctypes.c_int64), _p(offsets, ctypes.c_int64), 8)
        j = it.value
        return dict(x=x, iters=j, status=st, res=res[: j + 1])

    def geo_view(self) -> np.ndarray:
        """Geometric factors as [E, 7, Np] (rr, rs, rt, ss, st, tt, c)."""
        return self.geo.reshape(self.E, 7, self.Np)
