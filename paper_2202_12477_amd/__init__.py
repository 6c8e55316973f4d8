"""Python binding of libhbmi (include/hbmi.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
torch device tensors into device pointers and the current HIP stream into a
stream handle, and turns status codes into exceptions.  If libhbmi.so has not
been built the import still succeeds, but the first call raises: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhbmi.so")

HB_OK = 0
HB_ERR_INVALID_ARG = 1
HB_ERR_OUT_OF_MEMORY = 2
HB_ERR_DEVICE = 3
HB_ERR_NOT_CONVERGED = 4
HB_ERR_BREAKDOWN = 5
HB_ERR_NONFINITE = 6
HB_ERR_BUDGET = 7
HB_ERR_BUSY = 8

MASS_GWJ = 0
MASS_INVDEG = 1
MESH_FP32 = 1
MESH_DIRICHLET = 2
MESH_GATHER = 4
PREC_FP64 = 0
PREC_FP32_IR = 1
PREC_FP32_RR = 2
PRECOND_NONE = 0
PRECOND_JACOBI = 1

# Every entry point of include/hbmi.h, in declaration order.
EXPORTS = (
    "hb_mesh_create", "hb_mesh_destroy", "hb_mesh_query", "hb_mesh_export", "hb_rhs_uniform", "hb_ax", "hb_ax_add",
    "hb_ax_f32", "hb_cg_solve", "hb_cg_solve_noalloc", "hb_batch_solve", "hb_engine_footprint", "hb_engine_create", "hb_engine_destroy",
    "hb_engine_submit", "hb_engine_step", "hb_engine_poll", "hb_get_schedule", "hb_set_schedule", "hb_autotune",
    "hb_stream_probe", "hb_status_string", "hb_last_error",
)


class HbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


class _MeshDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("N", ctypes.c_int32),
                ("jitter", ctypes.c_double), ("seed", ctypes.c_uint64), ("mass", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class _MeshInfo(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int64), ("n_local", ctypes.c_int64), ("n_global", ctypes.c_int64),
                ("N", ctypes.c_int32), ("reserved", ctypes.c_int32), ("device_bytes", ctypes.c_size_t)]


class _EngineOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("iters_per_step", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("max_quota", ctypes.c_int32), ("graphs", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("autotune", ctypes.c_int32)]


class _EngineInfo(ctypes.Structure):
    _fields_ = [("running", ctypes.c_int32), ("queued", ctypes.c_int32), ("completed", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("used_bytes", ctypes.c_size_t), ("admit_s", ctypes.c_double),
                ("iterate_s", ctypes.c_double), ("retire_s", ctypes.c_double)]


class _CgOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("fixed_iters", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("x0_zero", ctypes.c_int32), ("check_every", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("inner_rtol", ctypes.c_double), ("graph_k", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("persistent", ctypes.c_int32), ("autotune", ctypes.c_int32)]


class _CgResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("res0", ctypes.c_double),
                ("res", ctypes.c_double), ("bnorm", ctypes.c_double), ("outer_iters", ctypes.c_int32),
                ("fp64_iters", ctypes.c_int32), ("persistent_segments", ctypes.c_int32)]


NUM_SCHED = 32  # tile schedule values 0..31 (hb_tune_result.us)


class _TuneResult(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("candidates", ctypes.c_int32), ("us", ctypes.c_double * NUM_SCHED)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libhbmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_12477_amd.build` "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    # torch (which supplies device memory and streams) brings its own HIP runtime; loading it first
    # makes this library bind to that same runtime, so both see one device context
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "hb_mesh_create": [ctypes.POINTER(_MeshDesc), vp, ctypes.POINTER(vp)],
        "hb_mesh_destroy": [vp],
        "hb_mesh_query": [vp, ctypes.POINTER(_MeshInfo)],
        "hb_mesh_export": [vp, vp, vp, vp, vp, vp],
        "hb_rhs_uniform": [i64, u64, vp, vp],
        "hb_ax": [vp, f64, vp, vp, vp],
        "hb_ax_add": [vp, f64, vp, vp, vp],
        "hb_ax_f32": [vp, f64, vp, vp, vp],
        "hb_cg_solve": [vp, f64, vp, vp, ctypes.POINTER(_CgOpts), ctypes.POINTER(_CgResult), vp, vp],
        "hb_cg_solve_noalloc": [vp, f64, vp, vp, ctypes.POINTER(_CgOpts), ctypes.POINTER(_CgResult), vp, vp],
        "hb_batch_solve": [i32, vp, vp, vp, vp, ctypes.POINTER(_CgOpts), ctypes.POINTER(_CgResult), vp],
        "hb_stream_probe": [vp, vp, i64, vp],
        "hb_engine_footprint": [ctypes.POINTER(_MeshDesc), i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "hb_engine_create": [ctypes.POINTER(_EngineOpts), vp, ctypes.POINTER(vp)],
        "hb_engine_destroy": [vp],
        "hb_engine_submit": [vp, ctypes.POINTER(_MeshDesc), f64, u64, f64, ctypes.POINTER(ctypes.c_uint64)],
        "hb_engine_step": [vp, i32, ctypes.POINTER(_EngineInfo)],
        "hb_engine_poll": [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), vp, ctypes.POINTER(_CgResult)],
        "hb_get_schedule": [i32, i32, ctypes.POINTER(ctypes.c_int32)],
        "hb_set_schedule": [i32, i32, i32],
        "hb_autotune": [i32, i32, i64, i32, ctypes.POINTER(_TuneResult), vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = i32
    L.hb_status_string.argtypes = [i32]
    L.hb_status_string.restype = ctypes.c_char_p
    L.hb_last_error.argtypes = []
    L.hb_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _status_name(st: int) -> str:
    try:
        return lib().hb_status_string(st).decode()
    except Exception:  # library missing: still give a readable name
        return f"status {st}"


def _check(st: int, what: str, ok=(HB_OK,)):
    if st not in ok:
        raise HbError(st, f"{what}: {lib().hb_last_error().decode()}")
    return st


def _stream(stream) -> int | None:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t, dtype=None) -> int:
    import torch

    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


@dataclass
class CgResult:
    iters: int
    status: int
    res0: float
    res: float
    bnorm: float
    outer_iters: int = 0
    fp64_iters: int = 0
    history: "list[float] | None" = None
    persistent_segments: int = 0


class Mesh:
    """A device-resident box mesh (hb_mesh_create / hb_mesh_destroy)."""

    def __init__(self, nx: int, ny: int, nz: int, N: int, jitter: float = 0.0, seed: int = 0,
                 mass: int = MASS_GWJ, fp32: bool = False, dirichlet: bool = False, gather: bool = False,
                 stream=None):
        """dirichlet: the boundary nodes of the box carry no DOF (N_G = (nx N - 1)(ny N - 1)(nz N - 1));
        gather: the two-phase operator (local output, then a deterministic gather) for every FP64 call."""
        flags = (MESH_FP32 if fp32 else 0) | (MESH_DIRICHLET if dirichlet else 0) | (MESH_GATHER if gather else 0)
        d = _MeshDesc(nx, ny, nz, N, jitter, seed, mass, flags)
        h = ctypes.c_void_p()
        _check(lib().hb_mesh_create(ctypes.byref(d), _stream(stream), ctypes.byref(h)), "hb_mesh_create")
        self._h = h
        info = _MeshInfo()
        _check(lib().hb_mesh_query(h, ctypes.byref(info)), "hb_mesh_query")
        self.nx, self.ny, self.nz, self.N, self.dirichlet, self.gather = nx, ny, nz, N, dirichlet, gather
        self.E, self.NL, self.NG = info.n_elem, info.n_local, info.n_global

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("mesh destroyed")
        return self._h

    def device_bytes(self) -> int:
        info = _MeshInfo()
        _check(lib().hb_mesh_query(self.handle, ctypes.byref(info)), "hb_mesh_query")
        return int(info.device_bytes)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().hb_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export(self):
        """Host copies: (geo [E,7,Np] float64, map [E,Np] int32, D, xi, w) as numpy arrays."""
        import numpy as np

        n1 = self.N + 1
        geo = np.empty((self.E, 7, n1 ** 3))
        mp = np.empty((self.E, n1 ** 3), dtype=np.int32)
        D, xi, w = np.empty((n1, n1)), np.empty(n1), np.empty(n1)
        _check(lib().hb_mesh_export(self.handle, geo.ctypes.data, mp.ctypes.data, D.ctypes.data, xi.ctypes.data,
                                    w.ctypes.data), "hb_mesh_export")
        return geo, mp, D, xi, w

    def ax(self, lam: float, x, y, stream=None):
        """y = A x on the device (asynchronous on the stream)."""
        import torch

        if x.numel() != self.NG or y.numel() != self.NG:
            raise ValueError("vectors must have N_G entries")
        _check(lib().hb_ax(self.handle, lam, _ptr(x, torch.float64), _ptr(y, torch.float64), _stream(stream)), "hb_ax")
        return y

    def ax_add(self, lam: float, x, y, stream=None):
        """y += A x on the device (asynchronous on the stream)."""
        import torch

        if x.numel() != self.NG or y.numel() != self.NG:
            raise ValueError("vectors must have N_G entries")
        _check(lib().hb_ax_add(self.handle, lam, _ptr(x, torch.float64), _ptr(y, torch.float64), _stream(stream)),
               "hb_ax_add")
        return y

    def ax_f32(self, lam: float, x, y, stream=None):
        """y = A_32 x with the FP32 operator (x float64, y float32; mesh built with fp32=True)."""
        import torch

        if x.numel() != self.NG or y.numel() != self.NG:
            raise ValueError("vectors must have N_G entries")
        _check(lib().hb_ax_f32(self.handle, lam, _ptr(x, torch.float64), _ptr(y, torch.float32), _stream(stream)),
               "hb_ax_f32")
        return y

    def cg(self, lam: float, b, x, *, max_iter: int = 100, fixed_iters: bool = True, rtol: float = 0.0,
           x0_zero: bool = True, check_every: int = 0, history: bool = True, prec: int = PREC_FP64,
           max_outer: int = 0, inner_rtol: float = 0.0, graph_k: int = 0, precond: int = PRECOND_NONE,
           stream=None, raise_on=(HB_ERR_INVALID_ARG, HB_ERR_OUT_OF_MEMORY, HB_ERR_DEVICE)) -> CgResult:
        """Algorithm 1 on the device (prec=PREC_FP64), or FP64 refinement around the FP32-operator CG
        (prec=PREC_FP32_IR / PREC_FP32_RR); x holds the initial guess (unless x0_zero) and the result.
        graph_k > 0 replays a captured graph of graph_k iterations instead of launching each kernel;
        precond=PRECOND_JACOBI (FP64 only) preconditions with the assembled diagonal of A."""
        import torch

        if b.numel() != self.NG or x.numel() != self.NG:
            raise ValueError("vectors must have N_G entries")
        opts = _CgOpts(max_iter, int(fixed_iters), rtol, int(x0_zero), check_every, prec, max_outer, inner_rtol,
                       graph_k, precond)
        res = _CgResult()
        hist = (ctypes.c_double * (max_iter + 1))() if history else None
        st = lib().hb_cg_solve(self.handle, lam, _ptr(b, torch.float64), _ptr(x, torch.float64), ctypes.byref(opts),
                               ctypes.byref(res), hist, _stream(stream))
        if st in raise_on:
            _check(st, "hb_cg_solve")
        out = CgResult(res.iters, res.status, res.res0, res.res, res.bnorm, res.outer_iters, res.fp64_iters)
        if history:
            k = res.outer_iters if prec != PREC_FP64 else res.iters
            out.history = list(hist[: min(k, max_iter) + 1])
        return out

    def cg_noalloc(self, lam: float, b, x, *, max_iter: int = 100, fixed_iters: bool = True, rtol: float = 0.0,
                   x0_zero: bool = True, check_every: int = 0, history: bool = True, precond: int = PRECOND_NONE,
                   stream=None, raise_on=(HB_ERR_INVALID_ARG, HB_ERR_OUT_OF_MEMORY, HB_ERR_DEVICE)) -> CgResult:
        """FP64 CG as cg(), with the workspace in the library's static device buffer
        (hb_cg_solve_noalloc: no device allocation; calls overlapping on one GPU race)."""
        import torch

        if b.numel() != self.NG or x.numel() != self.NG:
            raise ValueError("vectors must have N_G entries")
        opts = _CgOpts(max_iter, int(fixed_iters), rtol, int(x0_zero), check_every, PREC_FP64, 0, 0.0, 0, precond)
        res = _CgResult()
        hist = (ctypes.c_double * (max_iter + 1))() if history else None
        st = lib().hb_cg_solve_noalloc(self.handle, lam, _ptr(b, torch.float64), _ptr(x, torch.float64),
                                       ctypes.byref(opts), ctypes.byref(res), hist, _stream(stream))
        if st in raise_on:
            _check(st, "hb_cg_solve_noalloc")
        out = CgResult(res.iters, res.status, res.res0, res.res, res.bnorm)
        if history:
            out.history = list(hist[: min(res.iters, max_iter) + 1])
        return out


def batch_solve(meshes, lams, bs, xs, *, max_iter: int = 100, fixed_iters: bool = False, rtol: float = 1e-8,
                x0_zero: bool = True, check_every: int = 0, prec: int = PREC_FP64, inner_rtol: float = 0.0,
                graph_k: int = 0, precond: int = PRECOND_NONE, persistent: bool = False, autotune: bool = False,
                stream=None, raise_on=(HB_ERR_INVALID_ARG, HB_ERR_OUT_OF_MEMORY, HB_ERR_DEVICE)):
    """Solve independent problems together (hb_batch_solve); returns (status, [CgResult]).
    graph_k > 0: segments of graph_k iterations replayed from captured graphs; persistent: each segment
    as one persistent launch holding every running problem (where their degrees and boxes allow);
    autotune: tile schedules of the batch's classes timed at the classes' sizes first."""
    import torch

    n = len(meshes)
    if not (len(lams) == len(bs) == len(xs) == n):
        raise ValueError("one lambda, b and x per mesh")
    for m, b, x in zip(meshes, bs, xs):
        if b.numel() != m.NG or x.numel() != m.NG:
            raise ValueError("vectors must have N_G entries")
    H = (ctypes.c_void_p * n)(*[m.handle.value for m in meshes])
    L = (ctypes.c_double * n)(*lams)
    B = (ctypes.c_void_p * n)(*[_ptr(b, torch.float64) for b in bs])
    X = (ctypes.c_void_p * n)(*[_ptr(x, torch.float64) for x in xs])
    R = (_CgResult * n)()
    opts = _CgOpts(max_iter, int(fixed_iters), rtol, int(x0_zero), check_every, prec, 0, inner_rtol, graph_k,
                   precond, int(persistent), int(autotune))
    st = lib().hb_batch_solve(n, H, L, B, X, ctypes.byref(opts), R, _stream(stream))
    if st in raise_on:
        _check(st, "hb_batch_solve")
    return st, [CgResult(r.iters, r.status, r.res0, r.res, r.bnorm, r.outer_iters, r.fp64_iters,
                         persistent_segments=r.persistent_segments) for r in R]


def request_footprint(nx: int, ny: int, nz: int, N: int, prec: int = PREC_FP64, max_iter: int = 100000,
                      dirichlet: bool = False) -> int:
    """Device bytes a request of this size holds while the engine has it admitted."""
    d = _MeshDesc(nx, ny, nz, N, 0.0, 0, MASS_GWJ, MESH_DIRICHLET if dirichlet else 0)
    out = ctypes.c_size_t()
    _check(lib().hb_engine_footprint(ctypes.byref(d), prec, max_iter, ctypes.byref(out)), "hb_engine_footprint")
    return int(out.value)


class Engine:
    """Continuous-batching serving engine (hb_engine_*)."""

    def __init__(self, hbm_budget: int, max_slots: int, prec: int = PREC_FP32_RR, max_iter: int = 100000,
                 iters_per_step: int = 25, inner_rtol: float = 0.0, max_quota: int = 0, graphs: bool = False,
                 precond: int = PRECOND_NONE, autotune: bool = False, stream=None):
        o = _EngineOpts(hbm_budget, max_slots, prec, max_iter, iters_per_step, inner_rtol, max_quota, int(graphs),
                        precond, int(autotune))
        h = ctypes.c_void_p()
        self._stream = _stream(stream)
        _check(lib().hb_engine_create(ctypes.byref(o), self._stream, ctypes.byref(h)), "hb_engine_create")
        self._h = h
        self._ng = {}

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().hb_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, nx, ny, nz, N, *, jitter=0.05, seed=0, lam=1.0, rhs_seed=0, rtol=1e-8, mass=MASS_GWJ,
               dirichlet=False) -> int:
        d = _MeshDesc(nx, ny, nz, N, jitter, seed, mass, MESH_DIRICHLET if dirichlet else 0)
        t = ctypes.c_uint64()
        _check(lib().hb_engine_submit(self._h, ctypes.byref(d), lam, rhs_seed, rtol, ctypes.byref(t)),
               "hb_engine_submit")
        k = -1 if dirichlet else 1
        self._ng[t.value] = (nx * N + k) * (ny * N + k) * (nz * N + k)
        return int(t.value)

    def step(self, iters: int = 0) -> dict:
        info = _EngineInfo()
        _check(lib().hb_engine_step(self._h, iters, ctypes.byref(info)), "hb_engine_step")
        return dict(running=info.running, queued=info.queued, completed=info.completed, used_bytes=info.used_bytes,
                    admit_s=info.admit_s, iterate_s=info.iterate_s, retire_s=info.retire_s)

    def poll(self, ticket: int, want_x: bool = True):
        """None while running, else (CgResult, x as numpy array or None)."""
        import numpy as np

        done = ctypes.c_int32()
        r = _CgResult()
        x = np.empty(self._ng[ticket]) if want_x else None
        _check(lib().hb_engine_poll(self._h, ticket, ctypes.byref(done), x.ctypes.data if want_x else None,
                                    ctypes.byref(r)), "hb_engine_poll")
        if not done.value:
            return None
        del self._ng[ticket]
        return CgResult(r.iters, r.status, r.res0, r.res, r.bnorm, r.outer_iters, r.fp64_iters), x


def rhs_uniform(b, seed: int, stream=None):
    """Fill a float64 device vector with the seeded U[-1,1) forcing."""
    import torch

    _check(lib().hb_rhs_uniform(b.numel(), seed, _ptr(b, torch.float64), _stream(stream)), "hb_rhs_uniform")
    return b


SCHED_COLS_LDS = 1
SCHED_WAVE = 2
SCHED_LEAN = 4
SCHED_MERGE = 8
SCHED_THREE = 16


def get_schedule(N: int, prec: int = PREC_FP64) -> int:
    """The operator tile schedule of a (degree, precision) class (hb_get_schedule)."""
    v = ctypes.c_int32()
    _check(lib().hb_get_schedule(N, prec, ctypes.byref(v)), "hb_get_schedule")
    return v.value


def set_schedule(N: int, prec: int, schedule: int):
    """Pin a class's tile schedule (hb_set_schedule)."""
    _check(lib().hb_set_schedule(N, prec, schedule), "hb_set_schedule")


def autotune(N: int, prec: int = PREC_FP64, local_nodes: int = 0, reps: int = 20, stream=None) -> dict:
    """Time every tile schedule of a class on a box of about `local_nodes` local nodes (0: 2^22)
    and keep the fastest (hb_autotune)."""
    r = _TuneResult()
    _check(lib().hb_autotune(N, prec, local_nodes, reps, ctypes.byref(r), _stream(stream)), "hb_autotune")
    return {"N": N, "prec": prec, "schedule": r.schedule, "candidates": r.candidates,
            "us": {v: round(r.us[v], 2) for v in range(NUM_SCHED) if r.us[v] >= 0}}


def stream_probe(inp, out, stream=None):
    """8:1 streaming probe: out[i] = sum_k inp[k*n + i]."""
    import torch

    n = out.numel()
    if inp.numel() != 8 * n:
        raise ValueError("inp must hold 8*n entries")
    _check(lib().hb_stream_probe(_ptr(inp, torch.float64), _ptr(out, torch.float64), n, _stream(stream)),
           "hb_stream_probe")
    return out
