"""ctypes binding of libibfe.so (include/ibfe.h).  Argument marshalling only:
every step of the time step runs in the HIP library."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibfe.so")

IBFE_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOCONV", -5: "ENONFINITE", -6: "ESINGULAR"}
FIELD_USTAR, FIELD_UIB, FIELD_PHI = 0, 1, 2
OP_MASS, OP_STIFF, OP_GRAD, OP_DIV, OP_ADVDIFF, OP_INTERP, OP_SPREAD = range(7)
FLAG_P, FLAG_F, FLAG_DU, FLAG_PDIR, FLAG_HANG = 1, 2, 4, 8, 32

u8p = C.POINTER(C.c_uint8)
dp = C.POINTER(C.c_double)
i64p = C.POINTER(C.c_int64)


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
                ("origin", C.c_double * 3), ("node_mask", u8p), ("bc_tag", u8p),
                ("refine_cell", u8p)]


class IB(C.Structure):
    _fields_ = [("M", C.c_int64), ("X", dp), ("dS", C.c_double), ("U_B", dp)]


class Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("dt", C.c_double),
                ("precision", C.c_int32), ("rtol", C.c_double), ("max_iters", C.c_int32),
                ("precond", C.c_int32), ("advection", C.c_int32), ("ib_rtol", C.c_double),
                ("viscous", C.c_int32), ("advdiff", C.c_int32),
                ("mass_precond", C.c_int32)]


class Inlet(C.Structure):
    _fields_ = [("K", C.c_int32), ("omega", C.c_double), ("n", C.c_int64), ("node_ids", i64p),
                ("shape", dp)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Alloc(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("s1_iters", C.c_int32),
                ("ib_iters", C.c_int32), ("s3_iters", C.c_int32), ("s4_iters", C.c_int32),
                ("s1_outer", C.c_int32), ("s3_outer", C.c_int32), ("s4_outer", C.c_int32),
                ("s1_res", C.c_double), ("ib_res", C.c_double), ("s3_res", C.c_double),
                ("s4_res", C.c_double), ("poisson_apply_ms", C.c_double),
                ("poisson_applies", C.c_int64), ("mass_apply_ms", C.c_double),
                ("mass_applies", C.c_int64), ("s1_restarts", C.c_int32), ("reserved_", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 120), ("total_ms", C.c_double), ("launches", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("grid", C.POINTER(Grid)), ("ib", C.POINTER(IB)), ("params", C.POINTER(Params)),
                ("inlet", C.POINTER(Inlet)), ("nsteps", C.c_int32), ("t0", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("error", C.c_int32), ("n_u", C.c_int64), ("n_p", C.c_int64),
                ("footprint", C.c_size_t), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("stats", Stats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "stats"}
        d["stats"] = self.stats.as_dict()
        return d


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3

# name -> (restype, argtypes); the full exported surface of include/ibfe.h
SIGNATURES = {
    "ibfe_plan_create": (C.c_int, [C.POINTER(Grid), C.POINTER(IB), C.POINTER(Params),
                                   C.POINTER(Inlet), C.POINTER(C.c_void_p)]),
    "ibfe_plan_sizes": (C.c_int, [C.c_void_p, i64p, i64p, i64p, i64p, i64p]),
    "ibfe_plan_node_ids": (C.c_int, [C.c_void_p, i64p]),
    "ibfe_plan_node_flags": (C.c_int, [C.c_void_p, u8p]),
    "ibfe_plan_destroy": (None, [C.c_void_p]),
    "ibfe_create": (C.c_int, [C.POINTER(Grid), C.POINTER(IB), C.POINTER(Params), C.POINTER(Inlet),
                              C.POINTER(Alloc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "ibfe_num_nodes": (C.c_int, [C.c_void_p, i64p, i64p]),
    "ibfe_get_node_ids": (C.c_int, [C.c_void_p, i64p, i64p]),
    "ibfe_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int]),
    "ibfe_step": (C.c_int, [C.c_void_p, C.c_int]),
    "ibfe_run_steady": (C.c_int, [C.c_void_p, C.c_double, C.c_int64, C.c_void_p, C.c_void_p]),
    "ibfe_set_points": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "ibfe_set_points_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "ibfe_set_points_noalloc_max_points": (C.c_int64, []),
    "ibfe_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, dp, C.c_int]),
    "ibfe_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "ibfe_checkpoint_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "ibfe_checkpoint_save": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ibfe_checkpoint_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ibfe_inject_breakdown": (C.c_int, [C.c_void_p, C.c_int]),
    "ibfe_set_kernel_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "ibfe_get_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(KernelTime), C.c_int32, C.POINTER(C.c_int32)]),
    "ibfe_set_kernel_timing_filter": (C.c_int, [C.c_void_p, C.c_char_p]),
    "ibfe_set_graphs": (C.c_int, [C.c_void_p, C.c_int]),
    "ibfe_get_field": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    "ibfe_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "ibfe_wall_shear": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "ibfe_destroy": (None, [C.c_void_p]),
    "ibfe_last_error": (C.c_char_p, []),
    "ibfe_request_footprint": (C.c_int, [C.POINTER(Request), C.POINTER(C.c_size_t)]),
    "ibfe_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)]),
    "ibfe_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), i64p]),
    "ibfe_server_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Result)]),
    "ibfe_server_wait": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.POINTER(Result)]),
    "ibfe_server_fetch": (C.c_int, [C.c_void_p, C.c_int64, dp, dp, i64p]),
    "ibfe_server_peak_concurrency": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "ibfe_server_set_batching": (C.c_int, [C.c_void_p, C.c_double]),
    "ibfe_server_batch_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                          C.POINTER(C.c_int32)]),
    "ibfe_server_destroy": (None, [C.c_void_p]),
    "ibfe_batcher_create": (C.c_int, [C.c_double, C.POINTER(C.c_void_p)]),
    "ibfe_attach_batcher": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ibfe_batcher_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int32)]),
    "ibfe_batcher_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


class IbfeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2007_02082_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Importing it first makes the dynamic loader bind this library to that same
    # runtime, so torch's allocator and streams and this library share one
    # runtime instance; loading this library first would put two in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != IBFE_OK:
        raise IbfeError(rc, load().ibfe_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray | None, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


class _Inputs:
    """Keeps the ctypes structs and the numpy buffers they point to alive."""

    def __init__(self, nx, ny, nz, h, origin, node_mask, bc_tag, X, dS, U_B, rho, mu, dt,
                 inlet_K, inlet_omega, inlet_ids, inlet_shape, precision=0, rtol=0.0,
                 max_iters=0, ib_rtol=0.0, precond=0, advection=0, refine_cell=None, viscous=0,
                 advdiff=0, mass_precond=1):
        self.mask = np.ascontiguousarray(node_mask, dtype=np.uint8)
        self.refine = None if refine_cell is None else np.ascontiguousarray(refine_cell, dtype=np.uint8)
        self.tag = None if bc_tag is None else np.ascontiguousarray(bc_tag, dtype=np.uint8)
        self.X = np.ascontiguousarray(np.asarray(X, np.float64).reshape(-1, 3))
        self.UB = None if U_B is None else np.ascontiguousarray(np.asarray(U_B, np.float64).reshape(-1, 3))
        self.ids = np.ascontiguousarray(inlet_ids, dtype=np.int64)
        self.shape = np.ascontiguousarray(inlet_shape, dtype=np.float64)
        self.grid = Grid(int(nx), int(ny), int(nz), float(h), (C.c_double * 3)(*map(float, origin)),
                         _ptr(self.mask, C.c_uint8), _ptr(self.tag, C.c_uint8),
                         _ptr(self.refine, C.c_uint8))
        self.ib = IB(self.X.shape[0], _ptr(self.X, C.c_double) if self.X.size else None, float(dS),
                     _ptr(self.UB, C.c_double))
        self.params = Params(float(rho), float(mu), float(dt), int(precision), float(rtol),
                             int(max_iters), int(precond), int(advection), float(ib_rtol), int(viscous),
                             int(advdiff), int(mass_precond))
        self.inlet = Inlet(int(inlet_K), float(inlet_omega), self.ids.size,
                           _ptr(self.ids, C.c_int64) if self.ids.size else None,
                           _ptr(self.shape, C.c_double) if self.shape.size else None)


def inputs_from_case(case, **kw) -> dict:
    """Keyword arguments for Plan/Solver from any object with the fields of a flow case."""
    return dict(nx=case.nx, ny=case.ny, nz=case.nz, h=case.h, origin=case.origin,
                node_mask=case.node_mask, bc_tag=case.bc_tag, X=case.X, dS=case.dS, U_B=case.U_B,
                rho=case.rho, mu=case.mu, dt=case.dt, inlet_K=case.inlet_K,
                inlet_omega=case.inlet_omega, inlet_ids=case.inlet_ids,
                inlet_shape=case.inlet_shape, refine_cell=getattr(case, "refine_cell", None), **kw)


class Plan:
    """Host-only set-up (ibfe_plan_*): derived sets and canonical order."""

    def __init__(self, **kw):
        lib = load()
        self._in = _Inputs(**kw)
        h = C.c_void_p()
        check(lib.ibfe_plan_create(C.byref(self._in.grid), C.byref(self._in.ib),
                                   C.byref(self._in.params), C.byref(self._in.inlet), C.byref(h)))
        self._h = h
        f = 1 if kw.get("refine_cell") is None else 2   # refined: the fine lattice
        self.N = (f * int(kw["nx"]) + 1) * (f * int(kw["ny"]) + 1) * (f * int(kw["nz"]) + 1)

    def sizes(self) -> dict:
        v = [C.c_int64() for _ in range(5)]
        check(load().ibfe_plan_sizes(self._h, *[C.byref(x) for x in v]))
        return dict(zip(["n_p", "n_free", "n_pfree", "n_kept_cells", "n_floating"], [x.value for x in v]))

    def node_ids(self) -> np.ndarray:
        out = np.empty(self.sizes()["n_p"], np.int64)
        check(load().ibfe_plan_node_ids(self._h, _ptr(out, C.c_int64)))
        return out

    def node_flags(self) -> np.ndarray:
        out = np.empty(self.N, np.uint8)
        check(load().ibfe_plan_node_flags(self._h, _ptr(out, C.c_uint8)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().ibfe_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _torch_allocator():
    """Device allocator callbacks backed by torch's caching allocator."""
    import torch

    dev = torch.cuda.current_device()

    @ALLOC_FN
    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
        except Exception:
            return None

    delete = torch.cuda.caching_allocator_delete

    @FREE_FN
    def _free(ptr, user):
        try:
            delete(ptr)
        except Exception:
            pass  # torch is already torn down at interpreter exit; the process releases the memory

    return Alloc(_alloc, _free, None), (_alloc, _free)


class Solver:
    """One flow problem on the current GPU (ibfe_create ... ibfe_destroy)."""

    def __init__(self, stream=None, torch_alloc: bool = True, **kw):
        lib = load()
        self._in = _Inputs(**kw)
        self._keep = None
        alloc = None
        if torch_alloc:
            a, self._keep = _torch_allocator()
            self._alloc = a
            alloc = C.byref(a)
        import torch

        self._dev = torch.cuda.current_device()
        if stream is None:
            # a stream of its own (default priority): the null stream cannot be captured
            # into graphs; device tensors passed in are ordered against the current stream
            self._stream = torch.cuda.Stream()
            stream = self._stream.cuda_stream
        else:
            self._stream = None
        h = C.c_void_p()
        check(lib.ibfe_create(C.byref(self._in.grid), C.byref(self._in.ib), C.byref(self._in.params),
                              C.byref(self._in.inlet), alloc, C.c_void_p(stream), C.byref(h)))
        self._h = h
        nu, npr = C.c_int64(), C.c_int64()
        check(lib.ibfe_num_nodes(h, C.byref(nu), C.byref(npr)))
        self.n_u, self.n_p = nu.value, npr.value
        self.M = self._in.X.shape[0]

    # -- helpers ---------------------------------------------------------------
    def _vec(self, x, n: int, what: str, writable: bool = False):
        """(keep-alive object, pointer, on_device) for n float64 values held by a numpy
        array (converted to a contiguous float64 copy when read-only use allows it) or
        a torch tensor (float64, contiguous, exactly n elements; a CUDA tensor must be
        on this solver's device).  Anything else raises ValueError before the library
        sees the pointer, so a short or mistyped buffer never reaches a kernel."""
        if isinstance(x, np.ndarray):
            if writable:
                if x.dtype != np.float64 or not x.flags.c_contiguous or not x.flags.writeable:
                    raise ValueError(f"{what}: need a writable C-contiguous float64 array")
            else:
                x = np.ascontiguousarray(x, np.float64)
            if x.size != n:
                raise ValueError(f"{what}: {x.size} values given, {n} expected")
            return x, C.c_void_p(x.ctypes.data), 0
        try:
            import torch
        except ImportError:  # pragma: no cover - torch is a dependency of the package
            torch = None
        if torch is None or not isinstance(x, torch.Tensor):
            raise ValueError(f"{what}: need a numpy array or a torch tensor, got {type(x).__name__}")
        if x.dtype != torch.float64:
            raise ValueError(f"{what}: tensor dtype {x.dtype}, float64 expected")
        if not x.is_contiguous():
            raise ValueError(f"{what}: tensor is not contiguous")
        if x.numel() != n:
            raise ValueError(f"{what}: {x.numel()} values given, {n} expected")
        if x.is_cuda and getattr(self, "_dev", None) is not None and x.device.index != self._dev:
            raise ValueError(f"{what}: tensor on cuda:{x.device.index}, solver on cuda:{self._dev}")
        return x, C.c_void_p(x.data_ptr()), 1 if x.is_cuda else 0

    def node_ids(self) -> np.ndarray:
        out = np.empty(self.n_u, np.int64)
        check(load().ibfe_get_node_ids(self._h, _ptr(out, C.c_int64), None))
        return out

    def _after_caller(self):
        """Order the library's stream after the caller's current stream (device inputs)."""
        if self._stream is not None:
            import torch
            self._stream.wait_stream(torch.cuda.current_stream())

    def _before_caller(self):
        """Order the caller's current stream after the library's stream (device outputs)."""
        if self._stream is not None:
            import torch
            torch.cuda.current_stream().wait_stream(self._stream)

    def set_graphs(self, enable: bool):
        check(load().ibfe_set_graphs(self._h, 1 if enable else 0))

    def set_state(self, u, p, t: float = 0.0):
        """u: 3 x n_u values (SoA), p: n_p values; both numpy arrays or both tensors of
        one kind (host or this solver's device)."""
        u, pu, du = self._vec(u, 3 * self.n_u, "u")
        p, pp, dp_ = self._vec(p, self.n_p, "p")
        if du != dp_:
            raise ValueError("u and p must both be host or both be device memory")
        if du:
            self._after_caller()
        check(load().ibfe_set_state(self._h, pu, pp, float(t), du))

    def step(self, n: int = 1):
        check(load().ibfe_step(self._h, int(n)))

    def set_points_noalloc(self, X, U_B=None):
        """set_points without device allocation: the rebuild's scratch comes from the
        library's per-GPU static array (at most set_points_noalloc_max_points() points)."""
        self._set_points(X, U_B, load().ibfe_set_points_noalloc)

    @staticmethod
    def set_points_noalloc_max_points() -> int:
        return int(load().ibfe_set_points_noalloc_max_points())

    def set_points(self, X, U_B=None):
        """Move the Lagrangian points to X (M x 3) with prescribed velocities U_B (None = 0);
        the IB operators are rebuilt on the device.  X and U_B are numpy arrays, or
        contiguous float64 CUDA tensors (read on the library's stream after the caller's)."""
        self._set_points(X, U_B, load().ibfe_set_points)

    def _set_points(self, X, U_B, fn):
        X, px, dx = self._vec(X, 3 * self.M, "X")
        pb, db = None, dx
        if U_B is not None:
            U_B, pb, db = self._vec(U_B, 3 * self.M, "U_B")
        if db != dx:
            raise ValueError("X and U_B must both be host or both be device memory")
        if dx:
            self._after_caller()
        check(fn(self._h, px, pb, dx))

    def run_steady(self, tol: float, max_steps: int):
        """Step until the step-to-step NRMSE of every velocity component is below tol
        (or max_steps steps); returns (steps taken, the last step's three NRMSE)."""
        steps = C.c_int64()
        nr = np.empty(3)
        check(load().ibfe_run_steady(self._h, float(tol), int(max_steps), C.byref(steps),
                                     C.c_void_p(nr.ctypes.data)))
        return steps.value, nr

    def get_state(self):
        u = np.empty(3 * self.n_u)
        p = np.empty(self.n_p)
        t = C.c_double()
        check(load().ibfe_get_state(self._h, C.c_void_p(u.ctypes.data), C.c_void_p(p.ctypes.data),
                                    C.byref(t), 0))
        return u.reshape(3, self.n_u), p, t.value

    def get_state_device(self, u, p):
        """Write the state into device tensors (3*n_u and n_p doubles) without a host copy."""
        u, pu, du = self._vec(u, 3 * self.n_u, "u")
        p, pp, dp_ = self._vec(p, self.n_p, "p")
        if not (du and dp_):
            raise ValueError("get_state_device writes CUDA tensors; use get_state for host arrays")
        t = C.c_double()
        self._after_caller()
        check(load().ibfe_get_state(self._h, pu, pp, C.byref(t), 1))
        self._before_caller()
        return t.value

    def field(self, which: int) -> np.ndarray:
        n = self.n_p if which == FIELD_PHI else 3 * self.n_u
        out = np.empty(n)
        check(load().ibfe_get_field(self._h, int(which), C.c_void_p(out.ctypes.data), 0))
        return out if which == FIELD_PHI else out.reshape(3, self.n_u)

    def wall_shear(self, normals: np.ndarray) -> np.ndarray:
        """(M, 3) wall shear stress at the Lagrangian points for the current velocity."""
        n, _, _ = self._vec(np.asarray(normals), 3 * self.M, "normals")
        n = n.reshape(-1, 3)
        out = np.empty_like(n)
        check(load().ibfe_wall_shear(self._h, C.c_void_p(n.ctypes.data), C.c_void_p(out.ctypes.data), 0))
        return out

    def apply(self, op: int, x: np.ndarray, precision: int = 0) -> np.ndarray:
        in_len = {OP_MASS: self.n_p, OP_STIFF: self.n_p, OP_GRAD: self.n_p, OP_DIV: 3 * self.n_u,
                  OP_ADVDIFF: 3 * self.n_u, OP_INTERP: 3 * self.n_u, OP_SPREAD: 3 * self.M}[op]
        x, _, _ = self._vec(np.asarray(x), in_len, "x")
        out_len = {OP_MASS: self.n_p, OP_STIFF: self.n_p, OP_GRAD: 3 * self.n_u, OP_DIV: self.n_p,
                   OP_ADVDIFF: 3 * self.n_u, OP_INTERP: 3 * self.M, OP_SPREAD: 3 * self.n_u}[op]
        y = np.empty(out_len)
        check(load().ibfe_apply(self._h, int(op), int(precision), C.c_void_p(x.ctypes.data),
                                C.c_void_p(y.ctypes.data), 0))
        return y

    def checkpoint(self) -> bytes:
        """The time-stepping state (u, p, t, step count and the solvers' warm starts)
        as bytes; load_checkpoint on a solver built from the same inputs continues
        bit for bit."""
        n = C.c_size_t()
        check(load().ibfe_checkpoint_size(self._h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(load().ibfe_checkpoint_save(self._h, buf, n))
        return buf.raw

    def load_checkpoint(self, data: bytes):
        buf = C.create_string_buffer(bytes(data), len(data))
        check(load().ibfe_checkpoint_load(self._h, buf, C.c_size_t(len(data))))

    def inject_breakdown(self, iteration: int):
        """Testing aid: the next tentative-velocity BiCGStab solve reports a breakdown at
        this iteration (0 cancels)."""
        check(load().ibfe_inject_breakdown(self._h, int(iteration)))

    def stats(self) -> dict:
        s = Stats()
        check(load().ibfe_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def set_kernel_timing(self, on: bool):
        check(load().ibfe_set_kernel_timing(self._h, 1 if on else 0))

    def set_kernel_timing_filter(self, kernel: str | None):
        """Time only this kernel's dispatches (None: all kernels)."""
        check(load().ibfe_set_kernel_timing_filter(self._h, None if kernel is None else kernel.encode()))

    def kernel_times(self) -> list:
        """[(kernel name, total ms, dispatches)] since timing was enabled, longest first."""
        n = C.c_int32()
        check(load().ibfe_get_kernel_times(self._h, None, 0, C.byref(n)))
        buf = (KernelTime * max(1, n.value))()
        check(load().ibfe_get_kernel_times(self._h, buf, n.value, C.byref(n)))
        return [(buf[i].name.decode(), buf[i].total_ms, buf[i].launches) for i in range(n.value)]

    def close(self):
        if getattr(self, "_h", None):
            load().ibfe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def request_footprint(**kw) -> int:
    """Device bytes a request reserves (host-only estimate)."""
    nsteps = kw.pop("nsteps", 1)
    inp = _Inputs(**kw)
    req = Request(C.pointer(inp.grid), C.pointer(inp.ib), C.pointer(inp.params), C.pointer(inp.inlet),
                  int(nsteps), 0.0)
    out = C.c_size_t()
    check(load().ibfe_request_footprint(C.byref(req), C.byref(out)))
    return out.value


class Batcher:
    """Joins the mass-correction Chebyshev launches of the attached solvers
    (ibfe_batcher_*); solvers stepping from different threads batch together."""

    def __init__(self, window_us: float = 100.0):
        h = C.c_void_p()
        check(load().ibfe_batcher_create(float(window_us), C.byref(h)))
        self._h = h

    def attach(self, solver):
        check(load().ibfe_attach_batcher(solver._h, self._h))

    @staticmethod
    def detach(solver):
        check(load().ibfe_attach_batcher(solver._h, None))

    def stats(self) -> dict:
        b, m, w = C.c_int64(), C.c_int64(), C.c_int32()
        check(load().ibfe_batcher_stats(self._h, C.byref(b), C.byref(m), C.byref(w)))
        return {"batches": b.value, "members": m.value, "widest": w.value}

    def close(self):
        if getattr(self, "_h", None):
            check(load().ibfe_batcher_destroy(self._h))
            self._h = None


class Server:
    """Continuous-batching server (ibfe_server_*): requests run concurrently in
    worker slots, each on its own HIP stream, admitted by device footprint."""

    def __init__(self, budget_bytes: int = 0, max_slots: int = 4, batch_window_us: float | None = None):
        lib = load()
        h = C.c_void_p()
        check(lib.ibfe_server_create(C.c_size_t(int(budget_bytes)), int(max_slots), C.byref(h)))
        self._h = h
        if batch_window_us is not None:
            check(lib.ibfe_server_set_batching(self._h, float(batch_window_us)))

    def batch_stats(self) -> dict:
        b, m, w = C.c_int64(), C.c_int64(), C.c_int32()
        check(load().ibfe_server_batch_stats(self._h, C.byref(b), C.byref(m), C.byref(w)))
        return {"batches": b.value, "members": m.value, "widest": w.value}

    def submit(self, nsteps: int, t0: float = 0.0, **kw) -> int:
        inp = _Inputs(**kw)
        req = Request(C.pointer(inp.grid), C.pointer(inp.ib), C.pointer(inp.params), C.pointer(inp.inlet),
                      int(nsteps), float(t0))
        rid = C.c_int64()
        check(load().ibfe_server_submit(self._h, C.byref(req), C.byref(rid)))
        return rid.value

    def poll(self, rid: int) -> dict:
        r = Result()
        check(load().ibfe_server_poll(self._h, int(rid), C.byref(r)))
        return r.as_dict()

    def wait(self, rid: int, timeout: float = -1.0) -> dict:
        r = Result()
        check(load().ibfe_server_wait(self._h, int(rid), float(timeout), C.byref(r)))
        return r.as_dict()

    def fetch(self, rid: int, n_u: int, n_p: int):
        u = np.empty(3 * n_u)
        p = np.empty(n_p)
        ids = np.empty(n_u, np.int64)
        check(load().ibfe_server_fetch(self._h, int(rid), _ptr(u, C.c_double), _ptr(p, C.c_double),
                                       _ptr(ids, C.c_int64)))
        return u.reshape(3, n_u), p, ids

    def peak_concurrency(self) -> int:
        v = C.c_int32()
        check(load().ibfe_server_peak_concurrency(self._h, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            load().ibfe_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
