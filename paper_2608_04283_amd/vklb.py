"""Python binding of the C ABI in include/vklb.h (argument marshalling only).

Every step of the method runs in the HIP kernels of libvklb.so. PyTorch, when
present, supplies the device workspace (a uint8 CUDA tensor) and the stream;
without it the library allocates the workspace itself. If libvklb.so is
missing or no GPU is visible, calls raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvklb.so")

OK, ERR_ARG, ERR_UNSUPPORTED, ERR_OOM, ERR_DEVICE, ERR_NONPHYSICAL, ERR_STATE = 0, -1, -2, -3, -4, -5, -6
SYSTEMS = {"sw": 0, "shallow_water": 0, "euler": 1, "mhd": 2, "linear": 3}
PRECISIONS = {"fp64": 0, "f64": 0, "fp32": 1, "f32": 1}
BCS = {"periodic": 0, "zero_gradient": 1, "outflow": 1, "characteristic": 2}
EQ_SETS = {"weighted": 0, "centered": 1, "discontinuous": 2}

EXPORTED = ["vklb_workspace_bytes", "vklb_create", "vklb_set_end", "vklb_init", "vklb_init_device", "vklb_step", "vklb_moments",
            "vklb_progress", "vklb_diagnostics", "vklb_state_bytes", "vklb_get_state", "vklb_set_state", "vklb_last_step_ms",
            "vklb_destroy", "vklb_status_str", "vklb_last_error", "vklb_pool_create", "vklb_pool_submit",
            "vklb_pool_run", "vklb_pool_poll", "vklb_pool_get_stats", "vklb_pool_destroy", "vklb_tune",
            "vklb_run_static", "vklb_stream_copy", "vklb_pool_autotune"]
STATIC_BYTES = 64 * 1024 * 1024  # VKLB_STATIC_BYTES


class VklbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class System(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("g", ctypes.c_double), ("gamma", ctypes.c_double),
                ("ch_factor", ctypes.c_double), ("adv", ctypes.c_double * 2)]


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int64 * 2), ("lo", ctypes.c_double * 2),
                ("hi", ctypes.c_double * 2)]


class Speed(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("nu", ctypes.c_double), ("xi", ctypes.c_double)]


class Equilibrium(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("k", ctypes.c_double), ("alpha_local", ctypes.c_int), ("set", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("basis", ctypes.c_int), ("band_rows", ctypes.c_int), ("graph_chunk", ctypes.c_int),
                ("strip_width", ctypes.c_int), ("halo_rows", ctypes.c_int), ("small_grid", ctypes.c_int),
                ("fold_partials", ctypes.c_int)]


class Diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("steps", ctypes.c_int64), ("xi", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("ch", ctypes.c_double), ("done", ctypes.c_int),
                ("nonphysical", ctypes.c_int), ("fail_step", ctypes.c_int64), ("fail_cell", ctypes.c_int64),
                ("totals", ctypes.c_double * 9), ("max_div_b", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("sys", System), ("lat", ctypes.c_int), ("grid", Grid), ("lambda_", Speed), ("omega", ctypes.c_double),
                ("bc", ctypes.c_int * 2), ("eq", Equilibrium), ("T", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("U0", ctypes.c_void_p), ("U_out", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("t", ctypes.c_double),
                ("steps", ctypes.c_int64), ("fail_step", ctypes.c_int64), ("fail_cell", ctypes.c_int64)]


class RunInfo(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("steps", ctypes.c_int64), ("fail_step", ctypes.c_int64),
                ("fail_cell", ctypes.c_int64), ("done", ctypes.c_int), ("nonphysical", ctypes.c_int)]


class PoolStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("resident", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t),
                ("graph_launches", ctypes.c_int64), ("graph_captures", ctypes.c_int64)]


class PoolTile(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n", ctypes.c_int64), ("size_class", ctypes.c_int), ("band_rows", ctypes.c_int),
                ("halo_rows", ctypes.c_int), ("step_us", ctypes.c_double)]


_lib = None


def lib():
    """Load libvklb.so (built by __graft_entry__.build()); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # PyTorch ships its own HIP runtime (same soname as the system one). Load
    # it first so that libvklb binds to that copy: two HIP/HSA runtimes in one
    # process do not share the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    L.vklb_workspace_bytes.argtypes = [ctypes.POINTER(System), ctypes.c_int, ctypes.POINTER(Grid), ctypes.c_int]
    L.vklb_workspace_bytes.restype = ctypes.c_size_t
    L.vklb_create.argtypes = [ctypes.POINTER(System), ctypes.c_int, ctypes.POINTER(Grid), ctypes.POINTER(Speed),
                              ctypes.c_double, ctypes.c_int * 2, ctypes.POINTER(Equilibrium), ctypes.c_int,
                              ctypes.POINTER(Options), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.vklb_set_end.argtypes = [vp, ctypes.c_double, ctypes.c_int64]
    L.vklb_init.argtypes = [vp, dp]
    L.vklb_init_device.argtypes = [vp, vp]
    L.vklb_step.argtypes = [vp, ctypes.c_int64]
    L.vklb_moments.argtypes = [vp, dp, dp, ctypes.POINTER(ctypes.c_int64)]
    L.vklb_progress.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)]
    L.vklb_diagnostics.argtypes = [vp, ctypes.POINTER(Diag)]
    L.vklb_state_bytes.argtypes = [vp]
    L.vklb_state_bytes.restype = ctypes.c_size_t
    L.vklb_get_state.argtypes = [vp, vp, dp, ctypes.POINTER(ctypes.c_int64)]
    L.vklb_set_state.argtypes = [vp, vp]
    L.vklb_last_step_ms.argtypes = [vp, dp]
    L.vklb_destroy.argtypes = [vp]
    L.vklb_destroy.restype = None
    L.vklb_status_str.argtypes = [ctypes.c_int]
    L.vklb_status_str.restype = ctypes.c_char_p
    L.vklb_last_error.argtypes = [vp]
    L.vklb_last_error.restype = ctypes.c_char_p
    L.vklb_pool_create.argtypes = [ctypes.c_size_t, ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.vklb_pool_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.vklb_pool_run.argtypes = [vp, ctypes.c_int]
    L.vklb_pool_poll.argtypes = [vp, ctypes.POINTER(Completion), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.vklb_pool_get_stats.argtypes = [vp, ctypes.POINTER(PoolStats)]
    L.vklb_pool_autotune.argtypes = [vp, ctypes.POINTER(Request), ctypes.c_int, ctypes.c_int, ctypes.POINTER(PoolTile),
                                     ctypes.POINTER(ctypes.c_int)]
    L.vklb_pool_autotune.restype = ctypes.c_int
    L.vklb_pool_destroy.argtypes = [vp]
    L.vklb_pool_destroy.restype = None
    L.vklb_tune.argtypes = [ctypes.POINTER(System), ctypes.c_int, ctypes.POINTER(Grid), ctypes.POINTER(Speed),
                            ctypes.c_double, ctypes.c_int * 2, ctypes.POINTER(Equilibrium), ctypes.c_int,
                            ctypes.POINTER(Options), dp, ctypes.c_int, vp, ctypes.POINTER(Options), dp]
    L.vklb_run_static.argtypes = [ctypes.POINTER(System), ctypes.c_int, ctypes.POINTER(Grid), ctypes.POINTER(Speed),
                                  ctypes.c_double, ctypes.c_int * 2, ctypes.POINTER(Equilibrium), ctypes.c_int,
                                  ctypes.c_double, ctypes.c_int64, vp, vp, vp, vp]
    L.vklb_run_static.restype = ctypes.c_int
    L.vklb_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp]
    L.vklb_stream_copy.restype = ctypes.c_int
    for name in ("vklb_pool_create", "vklb_pool_submit", "vklb_pool_run", "vklb_pool_poll", "vklb_pool_get_stats"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("vklb_create", "vklb_set_end", "vklb_init", "vklb_init_device", "vklb_step", "vklb_moments", "vklb_progress",
                 "vklb_diagnostics",
                 "vklb_get_state", "vklb_set_state", "vklb_last_step_ms", "vklb_tune"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _structs(problem):
    P = problem
    sysd = System(SYSTEMS[P.system], P.g, P.gamma, P.ch_factor, (ctypes.c_double * 2)(*P.adv))
    n = (int(P.n[0]), int(P.n[1]) if P.dim == 2 else 1)
    grid = Grid(P.dim, (ctypes.c_int64 * 2)(*n), (ctypes.c_double * 2)(*P.lo), (ctypes.c_double * 2)(*P.hi))
    speed = Speed(0 if P.xi_mode == "cfl" else 1, P.nu, P.xi)
    eq = Equilibrium(P.c, P.k, 1 if getattr(P, "alpha_norm", "global") == "local" else 0,
                     EQ_SETS[getattr(P, "eq_set", "weighted")])
    bc = (ctypes.c_int * 2)(BCS[P.bc[0]], BCS[P.bc[1] if len(P.bc) > 1 else P.bc[0]])
    lat = 0 if P.dim == 1 else 1
    return sysd, lat, grid, speed, eq, bc


def workspace_bytes(problem, precision="fp64") -> int:
    sysd, lat, grid, _, _, _ = _structs(problem)
    return int(lib().vklb_workspace_bytes(ctypes.byref(sysd), lat, ctypes.byref(grid), PRECISIONS[precision]))


def tune(problem, precision="fp32", steps=20, basis=0, stream=None):
    """Fastest tile shape for `problem` (vklb_tune): returns (options dict, us per step)."""
    import torch
    L = lib()
    sysd, lat, grid, speed, eq, bc = _structs(problem)
    U0 = np.ascontiguousarray(np.asarray(problem.U0, dtype=np.float64).reshape(problem.p, problem.cells))
    base = Options(int(basis), 0, 0, 0, 0)
    best = Options()
    us = ctypes.c_double()
    st = stream if stream is not None else torch.cuda.current_stream()
    r = L.vklb_tune(ctypes.byref(sysd), lat, ctypes.byref(grid), ctypes.byref(speed), float(problem.omega), bc,
                    ctypes.byref(eq), PRECISIONS[precision], ctypes.byref(base), _dp(U0), int(steps),
                    st.cuda_stream, ctypes.byref(best), ctypes.byref(us))
    if r != OK:
        raise VklbError(r, L.vklb_last_error(None).decode())
    return ({"basis": best.basis, "strip_width": best.strip_width, "band_rows": best.band_rows,
             "halo_rows": best.halo_rows, "graph_chunk": best.graph_chunk, "small_grid": best.small_grid}, us.value)


def run_static(problem, precision, n_steps, U0_dev_ptr, U_dev_ptr, info_dev_ptr=None, stream=None, T=None):
    """vklb_run_static: the whole solve (init, n_steps step launches, moments)
    in the library's fixed workspace, enqueued on `stream` (a torch stream, or
    an int hipStream_t; None: torch's current stream). The arrays are device
    pointers (FP64 SoA [p][cells]); info_dev_ptr points to device memory for
    one RunInfo (or None). T defaults to the problem's end time."""
    L = lib()
    sysd, lat, grid, speed, eq, bc = _structs(problem)
    if T is None:
        T = problem.T if problem.T is not None else math.inf
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    sptr = stream if isinstance(stream, int) else stream.cuda_stream
    r = L.vklb_run_static(ctypes.byref(sysd), lat, ctypes.byref(grid), ctypes.byref(speed), float(problem.omega), bc,
                          ctypes.byref(eq), PRECISIONS[precision], float(T), int(n_steps),
                          ctypes.c_void_p(int(U0_dev_ptr)) if U0_dev_ptr else None,
                          ctypes.c_void_p(int(U_dev_ptr)) if U_dev_ptr else None,
                          ctypes.c_void_p(int(info_dev_ptr)) if info_dev_ptr else None, ctypes.c_void_p(sptr))
    if r != OK:
        raise VklbError(r, L.vklb_last_error(None).decode())


def stream_copy(dst_ptr, src_ptr, nbytes, non_temporal=True, stream=None):
    """vklb_stream_copy: the library's streaming copy kernel (device pointers)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    r = lib().vklb_stream_copy(ctypes.c_void_p(int(dst_ptr)), ctypes.c_void_p(int(src_ptr)), int(nbytes),
                               1 if non_temporal else 0, ctypes.c_void_p(st.cuda_stream))
    if r != OK:
        raise VklbError(r, lib().vklb_last_error(None).decode())


def stream_copy_bench(nbytes, reps=5):
    """Copy ceiling: HIP-event time of `reps` streaming copies of nbytes
    (after one warm-up) in both load/store forms; GB/s counts the bytes read
    plus the bytes written."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    out = {"bytes_per_copy": nbytes, "reps": reps}
    for nt in (True, False):
        stream_copy(b.data_ptr(), a.data_ptr(), nbytes, nt, st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            stream_copy(b.data_ptr(), a.data_ptr(), nbytes, nt, st)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out["non_temporal" if nt else "plain"] = {"ms_per_copy": round(ms, 4),
                                                  "gb_per_s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}
    del a, b
    return out


class Solver:
    """One WU-VKLB solve on the GPU (see include/vklb.h for the semantics)."""

    def __init__(self, problem, precision="fp64", basis=0, band_rows=0, graph_chunk=0, strip_width=0,
                 stream=None, use_torch=True, halo_rows=0, small_grid=0, fold_partials=0):
        self.problem = problem
        self.precision = precision
        self.p = problem.p
        self.cells = problem.cells
        L = lib()
        sysd, lat, grid, speed, eq, bc = _structs(problem)
        nbytes = workspace_bytes(problem, precision)
        if nbytes == 0:
            raise VklbError(ERR_ARG, "invalid problem for vklb_workspace_bytes")
        self._buf = None
        ptr = None
        sptr = None
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise VklbError(ERR_DEVICE, "no GPU visible to torch")
            self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self._buf.data_ptr()
            ptr = (base + 255) // 256 * 256
            st = stream if stream is not None else torch.cuda.current_stream()
            sptr = st.cuda_stream
            self._stream = st
        opt = Options(int(basis), int(band_rows), int(graph_chunk), int(strip_width), int(halo_rows),
                      int(small_grid), int(fold_partials))
        h = ctypes.c_void_p()
        r = L.vklb_create(ctypes.byref(sysd), lat, ctypes.byref(grid), ctypes.byref(speed), float(problem.omega), bc,
                          ctypes.byref(eq), PRECISIONS[precision], ctypes.byref(opt), ptr, nbytes, sptr,
                          ctypes.byref(h))
        if r != OK:
            raise VklbError(r, L.vklb_last_error(None).decode())
        self._h = h
        self.workspace_bytes = nbytes
        T = problem.T if problem.T is not None else math.inf
        self._check(L.vklb_set_end(self._h, float(T), int(min(problem.max_steps, 2**62))))

    def _check(self, r):
        if r != OK:
            raise VklbError(r, lib().vklb_last_error(self._h).decode() or lib().vklb_status_str(r).decode())
        return r

    def set_end(self, T=math.inf, max_steps=-1):
        """End condition (vklb_set_end): time T and/or a step count; after init
        it applies from the next step on, also to a solve that had finished."""
        self._check(lib().vklb_set_end(self._h, float(T), int(max_steps)))
        return self

    def init(self, U0=None):
        U0 = self.problem.U0 if U0 is None else U0
        U0 = np.ascontiguousarray(np.asarray(U0, dtype=np.float64).reshape(self.p, self.cells))
        self._check(lib().vklb_init(self._h, _dp(U0)))
        return self

    def init_device(self, U0_dev_ptr: int):
        """Initialize from an FP64 SoA array already in device memory (pointer)."""
        self._check(lib().vklb_init_device(self._h, ctypes.c_void_p(int(U0_dev_ptr))))
        return self

    def step(self, n: int):
        self._check(lib().vklb_step(self._h, int(n)))
        return self

    def moments(self):
        U = np.empty((self.p, self.cells), dtype=np.float64)
        t = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib().vklb_moments(self._h, _dp(U), ctypes.byref(t), ctypes.byref(n)))
        return U, t.value, n.value

    def diagnostics(self) -> dict:
        d = Diag()
        self._check(lib().vklb_diagnostics(self._h, ctypes.byref(d)))
        return {"t": d.t, "steps": d.steps, "xi": d.xi, "lambda_max": d.lambda_max, "ch": d.ch, "done": d.done,
                "nonphysical": d.nonphysical, "fail_step": d.fail_step, "fail_cell": d.fail_cell,
                "totals": np.array(d.totals[: self.p]), "max_div_b": d.max_div_b}

    def state_bytes(self) -> int:
        return int(lib().vklb_state_bytes(self._h))

    def get_state(self):
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        t = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib().vklb_get_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t),
                                         ctypes.byref(n)))
        return buf, t.value, n.value

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        if buf.nbytes != self.state_bytes():
            raise VklbError(ERR_ARG, "checkpoint size does not match this solver")
        self._check(lib().vklb_set_state(self._h, buf.ctypes.data_as(ctypes.c_void_p)))

    def last_step_ms(self) -> float:
        ms = ctypes.c_double()
        self._check(lib().vklb_last_step_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def progress(self):
        """(t, steps, done); synchronizes."""
        t = ctypes.c_double()
        n = ctypes.c_int64()
        d = ctypes.c_int()
        self._check(lib().vklb_progress(self._h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(d)))
        return t.value, n.value, bool(d.value)

    def run(self, steps=None, chunk=4096):
        """Run `steps` steps, or to the end condition when steps is None
        (enqueued in chunks, checking completion between them); returns (U, t, n)."""
        if steps is not None:
            self.step(steps)
            return self.moments()
        P = self.problem
        if P.max_steps < 2**62:
            self.step(int(P.max_steps))
            return self.moments()
        while True:
            self.step(chunk)
            _, _, done = self.progress()
            if done:
                return self.moments()

    def close(self):
        if getattr(self, "_h", None):
            lib().vklb_destroy(self._h)
            self._h = None
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Serving pool (vklb_pool_*): continuous batching of many solves."""

    def __init__(self, budget_bytes, precision="fp32", stream=None, use_torch=True):
        L = lib()
        sptr = None
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise VklbError(ERR_DEVICE, "no GPU visible to torch")
            st = stream if stream is not None else torch.cuda.current_stream()
            sptr = st.cuda_stream
        h = ctypes.c_void_p()
        r = L.vklb_pool_create(int(budget_bytes), PRECISIONS[precision], sptr, ctypes.byref(h))
        if r != OK:
            raise VklbError(r, "vklb_pool_create failed")
        self._h = h
        self._live = {}   # ticket -> (problem, U0, U_out)

    def _request(self, problem, U0, Uo, tag):
        sysd, lat, grid, speed, eq, bc = _structs(problem)
        T = problem.T if problem.T is not None else math.inf
        ms = int(problem.max_steps) if problem.max_steps < 2**62 else -1
        return Request(sysd, lat, grid, speed, float(problem.omega), bc, eq, float(T), ms,
                       U0.ctypes.data_as(ctypes.c_void_p), Uo.ctypes.data_as(ctypes.c_void_p), int(tag))

    def autotune(self, problems, steps=20):
        """vklb_pool_autotune over sample problems (their 2D ones); returns the
        tuned shapes as dicts. Call before the first submit."""
        keep = []
        reqs = (Request * max(1, len(problems)))()
        for i, P in enumerate(problems):
            U0 = np.ascontiguousarray(np.asarray(P.U0, dtype=np.float64).reshape(P.p, P.cells))
            Uo = np.empty_like(U0)
            keep.append((U0, Uo))
            reqs[i] = self._request(P, U0, Uo, i)
        out = (PoolTile * max(1, len(problems)))()
        n = ctypes.c_int(len(problems))
        r = lib().vklb_pool_autotune(self._h, reqs, len(problems), int(steps), out, ctypes.byref(n))
        if r != OK:
            raise VklbError(r, "vklb_pool_autotune failed")
        return [{f: getattr(out[i], f) for f, _ in PoolTile._fields_} for i in range(n.value)]

    def submit(self, problem, tag=0):
        sysd, lat, grid, speed, eq, bc = _structs(problem)
        U0 = np.ascontiguousarray(np.asarray(problem.U0, dtype=np.float64).reshape(problem.p, problem.cells))
        Uo = np.empty_like(U0)
        T = problem.T if problem.T is not None else math.inf
        ms = int(problem.max_steps) if problem.max_steps < 2**62 else -1
        rq = Request(sysd, lat, grid, speed, float(problem.omega), bc, eq, float(T), ms,
                     U0.ctypes.data_as(ctypes.c_void_p), Uo.ctypes.data_as(ctypes.c_void_p), int(tag))
        t = ctypes.c_uint64()
        r = lib().vklb_pool_submit(self._h, ctypes.byref(rq), ctypes.byref(t))
        if r != OK:
            raise VklbError(r, "vklb_pool_submit failed")
        self._live[t.value] = (problem, U0, Uo)
        return t.value

    def run(self, rounds):
        r = lib().vklb_pool_run(self._h, int(rounds))
        if r != OK:
            raise VklbError(r, "vklb_pool_run failed")

    def poll(self, max_items=4096):
        buf = (Completion * max_items)()
        n = ctypes.c_int()
        r = lib().vklb_pool_poll(self._h, buf, max_items, ctypes.byref(n))
        if r != OK:
            raise VklbError(r, "vklb_pool_poll failed")
        out = []
        for i in range(n.value):
            c = buf[i]
            prob, _, Uo = self._live.pop(c.ticket)
            out.append({"ticket": c.ticket, "tag": c.tag, "status": c.status, "t": c.t, "steps": c.steps,
                        "fail_step": c.fail_step, "fail_cell": c.fail_cell, "U": Uo, "problem": prob})
        return out

    def stats(self):
        st = PoolStats()
        lib().vklb_pool_get_stats(self._h, ctypes.byref(st))
        return {f: getattr(st, f) for f, _ in PoolStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().vklb_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
