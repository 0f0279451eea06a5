"""Python binding of libpgrad.so (argument marshalling only).

Every entry point of the C ABI (include/pgrad.h) is reachable under the same
name through :func:`lib`; the classes below own a plan and its workspace and
pass torch tensors' device pointers and the current HIP stream.  All the
arithmetic happens in the library's HIP kernels: if the library is missing
or cannot be loaded, every call raises :class:`PgError` -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpgrad.so")

# pg_status
OK, EINVAL, ERANGE, EDTYPE, EALIAS, EWORKSPACE, EHIP, EUNSUPPORTED, ESTATE = range(9)
STATUS_NAMES = ["PG_OK", "PG_EINVAL", "PG_ERANGE", "PG_EDTYPE", "PG_EALIAS", "PG_EWORKSPACE",
                "PG_EHIP", "PG_EUNSUPPORTED", "PG_ESTATE"]
F64, F32 = 0, 1
ADJ_AUTO, ADJ_ATOMIC, ADJ_GATHER, ADJ_COLOUR, ADJ_TILED = 0, 1, 2, 3, 4
RECOMPUTE, STORE, CKPT_AUTO = 0, 1, 2
WORKSPACE_ALIGN = 256

ADJOINTS = {"auto": ADJ_AUTO, "atomic": ADJ_ATOMIC, "gather": ADJ_GATHER, "colour": ADJ_COLOUR,
            "tiled": ADJ_TILED}
CKPTS = {"recompute": RECOMPUTE, "store": STORE, "auto": CKPT_AUTO}
EXPORT_CSR_OFFS, EXPORT_CSR_INC, EXPORT_COLOUR_OFFS, EXPORT_COLOUR_ELEMS = 0, 1, 2, 3

EXPORTS = ("pg_default_options", "pg_mesh_plan", "pg_dense_plan", "pg_bdense_plan",
           "pg_mesh_batch_plan", "pg_workspace_size", "pg_bind_workspace", "pg_objective",
           "pg_gradient", "pg_adjoint", "pg_hvp", "pg_jvp", "pg_timing", "pg_timing_read",
           "pg_tape_bytes", "pg_objective_tape", "pg_adjoint_tape", "pg_scale", "pg_plan_info",
           "pg_plan_export",
           "pg_laplace1d_plan", "pg_laplace1d_objective", "pg_laplace1d_gradient",
           "pg_plan_destroy", "pg_last_error", "pg_version",
           "pg_prog_create", "pg_prog_input", "pg_prog_const", "pg_prog_scale", "pg_prog_stencil",
           "pg_prog_gather", "pg_prog_add", "pg_prog_mul", "pg_prog_map", "pg_prog_scan",
           "pg_prog_segment_sum", "pg_prog_broadcast",
           "pg_prog_sum", "pg_prog_fusion", "pg_prog_plan", "pg_prog_bind_workspace", "pg_prog_run",
           "pg_prog_info", "pg_prog_destroy", "pg_mesh_gradient_noalloc")
MAPS = {"square": 0, "psi": 1}


class PgError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str = ""):
        name = STATUS_NAMES[code] if 0 <= code < len(STATUS_NAMES) else str(code)
        super().__init__(f"{where}: {name}: {msg}")
        self.code = code


class ProgStats(ctypes.Structure):
    _fields_ = [("fwd_kernels", ctypes.c_int32), ("rev_kernels", ctypes.c_int32),
                ("atomic_ops", ctypes.c_int32), ("rescheduled_ops", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("fused_gathers", ctypes.c_int32),
                ("dead_ops", ctypes.c_int32), ("folded_ops", ctypes.c_int32),
                ("tape_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64)]


class Options(ctypes.Structure):
    _fields_ = [("adjoint", ctypes.c_int32), ("ckpt", ctypes.c_int32), ("block", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("accumulate", ctypes.c_int32),
                ("scatter", ctypes.c_int32), ("onepass", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tape_budget", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("adjoint", ctypes.c_int32),
                ("ckpt", ctypes.c_int32), ("block", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("lds_slots", ctypes.c_int32), ("one_launch", ctypes.c_int32),
                ("n_colours", ctypes.c_int32), ("bound", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("tape_bytes", ctypes.c_int64),
                ("tape_budget", ctypes.c_int64)]


class Instance(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int64),
                ("node_off", ctypes.c_int64), ("elem_off", ctypes.c_int64)]


_lib = None
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZP = ctypes.POINTER(ctypes.c_size_t)
_PLANP = ctypes.POINTER(ctypes.c_void_p)


def lib():
    """Load libpgrad.so (built by paper_2507_13204_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PgError(EHIP, "load", f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2507_13204_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    L.pg_default_options.restype = Options
    L.pg_default_options.argtypes = []
    OP = ctypes.POINTER(Options)
    L.pg_mesh_plan.argtypes = [_PLANP, _I64, _I64, _I32, _VP, _VP, _VP, ctypes.c_int, OP, _SZP]
    L.pg_dense_plan.argtypes = [_PLANP, _I64, _I64, _VP, _VP, ctypes.c_int, OP, _SZP]
    L.pg_bdense_plan.argtypes = [_PLANP, _I64, _I64, _VP, _VP, ctypes.c_int, OP, _SZP]
    L.pg_mesh_batch_plan.argtypes = [_PLANP, _I32, ctypes.POINTER(Instance), _I32, _VP, _VP, _VP,
                                     ctypes.c_int, OP, _SZP]
    L.pg_workspace_size.argtypes = [_VP, _SZP]
    L.pg_bind_workspace.argtypes = [_VP, _VP, ctypes.c_size_t, _VP]
    L.pg_objective.argtypes = [_VP, _VP, _VP, _VP]
    L.pg_gradient.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.pg_adjoint.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.pg_hvp.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.pg_jvp.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.pg_tape_bytes.argtypes = [_VP, _SZP]
    L.pg_objective_tape.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.pg_adjoint_tape.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.pg_scale.argtypes = [ctypes.c_int, _I64, _VP, _VP, _VP, _VP]
    L.pg_plan_info.argtypes = [_VP, ctypes.POINTER(PlanInfo)]
    L.pg_plan_export.argtypes = [_VP, _I32, _VP, ctypes.c_size_t, _SZP]
    L.pg_mesh_gradient_noalloc.argtypes = [_I64, _I64, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]
    L.pg_plan_destroy.argtypes = [_VP]
    L.pg_timing.argtypes = [_VP, _I32]
    L.pg_timing_read.argtypes = [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]
    L.pg_laplace1d_plan.argtypes = [_PLANP, _I64, ctypes.c_int, OP, _SZP]
    L.pg_laplace1d_objective.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.pg_laplace1d_gradient.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, _VP]
    I32P = ctypes.POINTER(_I32)
    D = ctypes.c_double
    L.pg_prog_create.argtypes = [_PLANP]
    L.pg_prog_input.argtypes = [_VP, _I64, I32P]
    L.pg_prog_const.argtypes = [_VP, _I64, _VP, I32P]
    L.pg_prog_scale.argtypes = [_VP, _I32, D, I32P]
    L.pg_prog_stencil.argtypes = [_VP, _I32, _I32, I32P, ctypes.POINTER(D), I32P]
    L.pg_prog_gather.argtypes = [_VP, _I32, _I64, _I32, _VP, _VP, I32P]
    L.pg_prog_add.argtypes = [_VP, _I32, D, _I32, D, I32P]
    L.pg_prog_mul.argtypes = [_VP, _I32, _I32, I32P]
    L.pg_prog_map.argtypes = [_VP, _I32, ctypes.c_int, I32P]
    L.pg_prog_scan.argtypes = [_VP, _I32, I32P]
    L.pg_prog_segment_sum.argtypes = [_VP, _I32, _I64, _VP, I32P]
    L.pg_prog_broadcast.argtypes = [_VP, _I32, _VP, _I64, I32P]
    L.pg_prog_sum.argtypes = [_VP, _I32]
    L.pg_prog_plan.argtypes = [_VP, _SZP]
    L.pg_prog_bind_workspace.argtypes = [_VP, _VP, ctypes.c_size_t]
    L.pg_prog_run.argtypes = [_VP, ctypes.POINTER(_VP), _VP, ctypes.POINTER(_VP), _VP, _VP]
    L.pg_prog_fusion.argtypes = [_VP, _I32]
    L.pg_prog_info.argtypes = [_VP, ctypes.POINTER(ProgStats)]
    L.pg_prog_destroy.argtypes = [_VP]
    for name in EXPORTS:
        if name.startswith("pg_prog_"):
            getattr(L, name).restype = ctypes.c_int
    L.pg_last_error.restype = ctypes.c_char_p
    L.pg_last_error.argtypes = []
    L.pg_version.restype = ctypes.c_int
    L.pg_version.argtypes = []
    for name in ("pg_mesh_plan", "pg_dense_plan", "pg_bdense_plan", "pg_mesh_batch_plan",
                 "pg_workspace_size", "pg_bind_workspace", "pg_objective", "pg_gradient",
                 "pg_adjoint", "pg_hvp", "pg_jvp", "pg_timing", "pg_timing_read", "pg_plan_destroy",
                 "pg_tape_bytes", "pg_objective_tape", "pg_adjoint_tape", "pg_scale",
                 "pg_plan_info", "pg_plan_export", "pg_mesh_gradient_noalloc",
                 "pg_laplace1d_plan", "pg_laplace1d_objective", "pg_laplace1d_gradient"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(code: int, where: str):
    if code != OK:
        raise PgError(code, where, lib().pg_last_error().decode(errors="replace"))


def make_options(adjoint="auto", ckpt="recompute", block: int = 0, tile: int = 0,
                 accumulate: bool = False, scatter: int = 0, onepass: bool = True,
                 tape_budget: int = 0) -> Options:
    o = Options()
    o.adjoint = ADJOINTS[adjoint] if isinstance(adjoint, str) else int(adjoint)
    o.ckpt = CKPTS[ckpt] if isinstance(ckpt, str) else int(ckpt)
    o.block = int(block)
    o.tile = int(tile)
    o.accumulate = int(bool(accumulate))
    o.scatter = int(scatter)
    o.onepass = 0 if onepass else 1
    o.reserved = 0
    o.tape_budget = int(tape_budget)
    return o


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise PgError(EDTYPE, "dtype", f"unsupported tensor dtype {t.dtype}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(stream=None):
    if stream is None:
        if _raw_stream is not None:  # the current stream's handle without a Stream object
            return ctypes.c_void_p(_raw_stream(torch.cuda.current_device()))
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise PgError(EINVAL, "tensor", "operands must be contiguous CUDA (HIP) tensors")


class _Plan:
    """Owns a pg_plan and the workspace tensor bound to it."""

    def __init__(self):
        self._plan = ctypes.c_void_p()
        self._ws = None
        self.workspace_bytes = 0

    def _bind(self, device, stream=None):
        nbytes = self.workspace_bytes
        if nbytes > 0:
            raw = torch.empty(nbytes + WORKSPACE_ALIGN, dtype=torch.uint8, device=device)
            off = (-raw.data_ptr()) % WORKSPACE_ALIGN
            self._ws_raw = raw
            self._ws = raw[off:off + nbytes]
            ptr = ctypes.c_void_p(self._ws.data_ptr())
        else:
            ptr = None
        check(lib().pg_bind_workspace(self._plan, ptr, nbytes, _stream(stream)), "pg_bind_workspace")

    def close(self):
        if self._plan:
            lib().pg_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        """pg_plan_info: the plan's resolved choices (ckpt, adjoint, LDS table, ...)."""
        st = PlanInfo()
        check(lib().pg_plan_info(self._plan, ctypes.byref(st)), "pg_plan_info")
        return {name: getattr(st, name) for name, _ in PlanInfo._fields_}

    def tape_bytes(self) -> int:
        sz = ctypes.c_size_t()
        check(lib().pg_tape_bytes(self._plan, ctypes.byref(sz)), "pg_tape_bytes")
        return sz.value

    def new_tape(self, device) -> torch.Tensor:
        """A caller-owned tape for one forward pass (pg_objective_tape)."""
        n = self.tape_bytes()
        return torch.empty((n + 15) // 16 * 2, dtype=torch.float64, device=device)

    def objective_tape(self, x, tape, f_shape=(), stream=None, f_out=None):
        _need_cuda(x, tape)
        f = torch.empty(f_shape, dtype=torch.float64, device=x.device) if f_out is None else f_out
        check(lib().pg_objective_tape(self._plan, _ptr(x), _ptr(f), _ptr(tape), _stream(stream)),
              "pg_objective_tape")
        return f

    def adjoint_tape(self, fbar, tape, like, out=None, stream=None):
        _need_cuda(fbar, tape, out)
        g = torch.empty_like(like) if out is None else out
        check(lib().pg_adjoint_tape(self._plan, _ptr(fbar), _ptr(tape), _ptr(g), _stream(stream)),
              "pg_adjoint_tape")
        return g

    # What the forward of an autograd Function keeps for its backward:
    #   "gradient":  f and the gradient in one pg_gradient call; the backward
    #                scales the saved gradient by grad_output (pg_scale);
    #   "store":     the forward values on a per-call tape (pg_objective_tape);
    #   "recompute": nothing; the backward recomputes them (pg_adjoint).
    # "auto" takes the first of these whose saved bytes fit the budget
    # (autograd_budget bytes, or a quarter of the free device memory when the
    # objective is made).
    _POLICIES = ("gradient", "store", "recompute")

    def _resolve_autograd(self, policy, budget, x_bytes, device, allowed):
        if policy != "auto":
            if policy not in allowed:
                raise PgError(EINVAL, "autograd", f"policy {policy!r} not offered here ({allowed})")
            return policy
        if not budget:
            free, _ = torch.cuda.mem_get_info(device)
            budget = free // 4
        self.autograd_budget = int(budget)
        saved = {"gradient": x_bytes,
                 "store": self.tape_bytes() if "store" in allowed else None}
        for pol in self._POLICIES:
            if pol not in allowed:
                continue
            if pol == "recompute" or saved[pol] <= budget:
                return pol
        return "recompute"

    def _stores_tape(self) -> bool:
        """True if the plan's resolved checkpoint is PG_STORE (pg_adjoint
        then reads the workspace tape of the last pg_objective)."""
        if getattr(self, "_stores", None) is None:
            self._stores = self.info()["ckpt"] == STORE
        return self._stores

    def timing(self, mode: int):
        """0 off, 1 time the dominant kernel of each call, 2 time each call."""
        check(lib().pg_timing(self._plan, int(mode)), "pg_timing")

    def timing_read(self) -> Tuple[float, int]:
        """(total milliseconds, number of timed launches) since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(lib().pg_timing_read(self._plan, ctypes.byref(ms), ctypes.byref(n)), "pg_timing_read")
        return ms.value, n.value

    # generic calls -----------------------------------------------------
    def _objective(self, x, f_shape, stream=None, f_out=None):
        f = torch.empty(f_shape, dtype=torch.float64, device=x.device) if f_out is None else f_out
        check(lib().pg_objective(self._plan, _ptr(x), _ptr(f), _stream(stream)), "pg_objective")
        return f

    def _gradient(self, x, f_shape, out=None, want_f=True, stream=None, f_out=None):
        g = torch.empty_like(x) if out is None else out
        f = f_out
        if f is None and want_f:
            f = torch.empty(f_shape, dtype=torch.float64, device=x.device)
        check(lib().pg_gradient(self._plan, _ptr(x), _ptr(g), _ptr(f), _stream(stream)),
              "pg_gradient")
        return f, g

    def _adjoint(self, x, fbar, out=None, stream=None):
        g = torch.empty_like(x) if out is None else out
        check(lib().pg_adjoint(self._plan, _ptr(x), _ptr(fbar), _ptr(g), _stream(stream)),
              "pg_adjoint")
        return g


class MeshObjective(_Plan):
    """f(x) = sum_e w_e psi(sum_j B[e,j] x[conn[e,j]]) and its gradient."""

    def __init__(self, conn: torch.Tensor, B: torch.Tensor, w: torch.Tensor, n_nodes: int,
                 adjoint="auto", ckpt="recompute", block: int = 0, tile: int = 0,
                 accumulate: bool = False, scatter: int = 0, onepass: bool = True, stream=None,
                 tape_budget: int = 0, autograd: str = "auto", autograd_budget: int = 0):
        super().__init__()
        _need_cuda(conn, B, w)
        if conn.dtype != torch.int32:
            raise PgError(EINVAL, "MeshObjective", "conn must be int32")
        E = conn.shape[0] if conn.dim() == 2 else 0
        k = conn.shape[1] if conn.dim() == 2 else 1
        self.conn, self.B, self.w = conn, B, w
        self.n_nodes, self.n_elems, self.k = int(n_nodes), int(E), int(k)
        self.dtype = B.dtype
        self.options = make_options(adjoint, ckpt, block, tile, accumulate, scatter, onepass,
                                    tape_budget)
        sz = ctypes.c_size_t()
        check(lib().pg_mesh_plan(ctypes.byref(self._plan), self.n_nodes, E, k, _ptr(conn),
                                 _ptr(B), _ptr(w), _dtype_code(B), ctypes.byref(self.options),
                                 ctypes.byref(sz)), "pg_mesh_plan")
        self.workspace_bytes = sz.value
        self._bind(conn.device, stream)
        self.autograd_budget = int(autograd_budget)
        self.autograd_policy = self._resolve_autograd(
            autograd, autograd_budget, self.n_nodes * B.element_size(), conn.device,
            ("gradient", "store", "recompute"))

    def export(self, what: int) -> "np.ndarray":
        """pg_plan_export: a bound plan's transposed connectivity or colour
        classes, copied to the host."""
        import numpy as np
        sz = ctypes.c_size_t()
        check(lib().pg_plan_export(self._plan, int(what), None, 0, ctypes.byref(sz)),
              "pg_plan_export")
        dt = np.int64 if what == EXPORT_COLOUR_OFFS else np.int32
        out = np.empty(sz.value // np.dtype(dt).itemsize, dtype=dt)
        check(lib().pg_plan_export(self._plan, int(what), out.ctypes.data_as(ctypes.c_void_p),
                                   out.nbytes, ctypes.byref(sz)), "pg_plan_export")
        return out

    def objective(self, x, stream=None, f_out=None):
        _need_cuda(x)
        return self._objective(x, (), stream, f_out)

    def gradient(self, x, out=None, want_f=True, stream=None, f_out=None):
        _need_cuda(x, out)
        return self._gradient(x, (), out, want_f, stream, f_out)

    def adjoint(self, x, fbar, out=None, stream=None):
        _need_cuda(x, fbar, out)
        return self._adjoint(x, fbar, out, stream)

    def hvp(self, x, v, out=None, stream=None):
        _need_cuda(x, v, out)
        h = torch.empty_like(x) if out is None else out
        check(lib().pg_hvp(self._plan, _ptr(x), _ptr(v), _ptr(h), _stream(stream)), "pg_hvp")
        return h

    def jvp(self, x, d, stream=None):
        """Directional derivative f'(x) . d (forward tangent), a 0-d FP64 tensor."""
        _need_cuda(x, d)
        out = torch.empty((), dtype=torch.float64, device=x.device)
        check(lib().pg_jvp(self._plan, _ptr(x), _ptr(d), _ptr(out), _stream(stream)), "pg_jvp")
        return out


class DenseObjective(_Plan):
    """f(x) = sum_i w_i psi((A x)_i) and its gradient."""

    def __init__(self, A: torch.Tensor, w: torch.Tensor, accumulate: bool = False, stream=None,
                 autograd: str = "auto", autograd_budget: int = 0):
        super().__init__()
        _need_cuda(A, w)
        self.A, self.w = A, w
        self.rows, self.cols = int(A.shape[0]), int(A.shape[1])
        self.options = make_options(accumulate=accumulate)
        sz = ctypes.c_size_t()
        check(lib().pg_dense_plan(ctypes.byref(self._plan), self.rows, self.cols, _ptr(A), _ptr(w),
                                  _dtype_code(A), ctypes.byref(self.options), ctypes.byref(sz)),
              "pg_dense_plan")
        self.workspace_bytes = sz.value
        self._bind(A.device, stream)
        self.autograd_budget = int(autograd_budget)
        self.autograd_policy = self._resolve_autograd(
            autograd, autograd_budget, self.cols * A.element_size(), A.device,
            ("gradient", "recompute"))

    def objective(self, x, stream=None, f_out=None):
        _need_cuda(x)
        return self._objective(x, (), stream, f_out)

    def gradient(self, x, out=None, want_f=True, stream=None, f_out=None):
        _need_cuda(x, out)
        return self._gradient(x, (), out, want_f, stream, f_out)

    def adjoint(self, x, fbar, out=None, stream=None):
        _need_cuda(x, fbar, out)
        return self._adjoint(x, fbar, out, stream)


class BatchedDense(_Plan):
    """f(X) = sum W (.) psi(A X) with both products on the matrix cores."""

    def __init__(self, A: torch.Tensor, W: torch.Tensor, ckpt="auto", accumulate: bool = False,
                 stream=None, tape_budget: int = 0, autograd: str = "auto",
                 autograd_budget: int = 0):
        super().__init__()
        _need_cuda(A, W)
        self.A, self.W = A, W
        self.m, self.n = int(W.shape[0]), int(W.shape[1])
        self.options = make_options(ckpt=ckpt, accumulate=accumulate, tape_budget=tape_budget)
        sz = ctypes.c_size_t()
        check(lib().pg_bdense_plan(ctypes.byref(self._plan), self.m, self.n, _ptr(A), _ptr(W),
                                   _dtype_code(A), ctypes.byref(self.options), ctypes.byref(sz)),
              "pg_bdense_plan")
        self.workspace_bytes = sz.value
        self._bind(A.device, stream)
        self.autograd_budget = int(autograd_budget)
        self.autograd_policy = self._resolve_autograd(
            autograd, autograd_budget, self.m * self.n * W.element_size(), A.device,
            ("gradient", "store", "recompute"))

    def objective(self, X, stream=None, f_out=None):
        _need_cuda(X)
        return self._objective(X, (), stream, f_out)

    def gradient(self, X, out=None, want_f=True, stream=None, f_out=None):
        _need_cuda(X, out)
        return self._gradient(X, (), out, want_f, stream, f_out)

    def adjoint(self, X, fbar, out=None, stream=None):
        _need_cuda(X, fbar, out)
        return self._adjoint(X, fbar, out, stream)


class MeshBatch(_Plan):
    """Many meshes in one launch (one workgroup per tile, largest instance
    first); per-instance objectives."""

    def __init__(self, inst, conn: torch.Tensor, B: torch.Tensor, w: torch.Tensor,
                 ckpt="recompute", block: int = 0, tile: int = 0, accumulate: bool = False,
                 scatter: int = 0, stream=None, tape_budget: int = 0, autograd: str = "auto",
                 autograd_budget: int = 0):
        super().__init__()
        _need_cuda(conn, B, w)
        self.conn, self.B, self.w = conn, B, w
        rows = [tuple(int(v) for v in r) for r in inst]
        self.n_inst = len(rows)
        arr = (Instance * max(self.n_inst, 1))()
        for i, (nn, ne, no, eo) in enumerate(rows):
            arr[i] = Instance(nn, ne, no, eo)
        self.n_nodes = max([r[0] + r[2] for r in rows], default=0)
        k = conn.shape[1] if conn.dim() == 2 else 8
        self.options = make_options("atomic", ckpt, block, tile, accumulate, scatter,
                                    tape_budget=tape_budget)
        sz = ctypes.c_size_t()
        check(lib().pg_mesh_batch_plan(ctypes.byref(self._plan), self.n_inst, arr, k, _ptr(conn),
                                       _ptr(B), _ptr(w), _dtype_code(B), ctypes.byref(self.options),
                                       ctypes.byref(sz)), "pg_mesh_batch_plan")
        self.workspace_bytes = sz.value
        self._bind(conn.device, stream)
        # per-instance seeds: the saved-gradient policy does not apply
        self.autograd_budget = int(autograd_budget)
        self.autograd_policy = self._resolve_autograd(
            autograd, autograd_budget, 0, conn.device, ("store", "recompute"))

    def objective(self, x, stream=None, f_out=None):
        _need_cuda(x)
        return self._objective(x, (self.n_inst,), stream, f_out)

    def gradient(self, x, out=None, want_f=True, stream=None, f_out=None):
        _need_cuda(x, out)
        return self._gradient(x, (self.n_inst,), out, want_f, stream, f_out)

    def adjoint(self, x, fbar, out=None, stream=None):
        _need_cuda(x, fbar, out)
        return self._adjoint(x, fbar, out, stream)


class Laplace1D(_Plan):
    """The paper's section 4 example: f(x, b) = ||A(3x) - b||^2, A the 1D
    Laplacian; gradients in x and b.  adjoint: 'gather' (default, rescheduled
    reverse threads) or 'atomic' (the paper's scatter schedule)."""

    def __init__(self, n: int, dtype=torch.float64, adjoint="gather", accumulate: bool = False,
                 device="cuda", stream=None):
        super().__init__()
        self.n = int(n)
        self.dtype = dtype
        code = F64 if dtype == torch.float64 else F32 if dtype == torch.float32 else -1
        self.options = make_options(adjoint=adjoint, accumulate=accumulate)
        sz = ctypes.c_size_t()
        check(lib().pg_laplace1d_plan(ctypes.byref(self._plan), self.n, code,
                                      ctypes.byref(self.options), ctypes.byref(sz)),
              "pg_laplace1d_plan")
        self.workspace_bytes = sz.value
        self._bind(torch.device(device), stream)

    def objective(self, x, b, stream=None, f_out=None):
        _need_cuda(x, b)
        f = torch.empty((), dtype=torch.float64, device=x.device) if f_out is None else f_out
        check(lib().pg_laplace1d_objective(self._plan, _ptr(x), _ptr(b), _ptr(f), _stream(stream)),
              "pg_laplace1d_objective")
        return f

    def gradient(self, x, b, gx=None, gb=None, want=("x", "b"), stream=None, f_out=None):
        _need_cuda(x, b, gx, gb)
        if gx is None and "x" in want:
            gx = torch.empty_like(x)
        if gb is None and "b" in want:
            gb = torch.empty_like(b)
        f = torch.empty((), dtype=torch.float64, device=x.device) if f_out is None else f_out
        check(lib().pg_laplace1d_gradient(self._plan, _ptr(x), _ptr(b), _ptr(gx), _ptr(gb),
                                          _ptr(f), _stream(stream)), "pg_laplace1d_gradient")
        return f, gx, gb


# ---------------------------------------------------------- composed programs

class Program:
    """A chain of data-parallel constructs ending in a sum, whose reverse pass
    the library generates construct by construct (pg_prog_* in the C ABI).

    Builders return view ids.  Device operands given to ``const`` and
    ``gather`` are kept referenced by this object.  ``plan(device)`` runs the
    activity analysis, lays out the tape and binds a workspace; ``run`` then
    evaluates f and, when asked, the gradient with respect to every input.
    """

    def __init__(self, fusion: int = 1):
        self._p = ctypes.c_void_p()
        check(lib().pg_prog_create(ctypes.byref(self._p)), "pg_prog_create")
        check(lib().pg_prog_fusion(self._p, int(fusion)), "pg_prog_fusion")
        self._keep = []
        self._ws = None
        self.n_inputs = 0
        self.input_lengths = []
        self.workspace_bytes = 0

    @classmethod
    def from_spec(cls, spec, device="cuda", fusion: int = 1) -> "Program":
        """Build (not plan) a program from construct tuples: ("input", n),
        ("const", data), ("scale", a, alpha), ("stencil", a, offsets, coeffs),
        ("gather", a, conn, B), ("add", a, alpha, b, beta), ("mul", a, b),
        ("map", a, fn), ("scan", a), ("segsum", a, offsets), ("bcast", a,
        offsets), ("sum", a); array operands (NumPy or
        torch) are copied to the device."""
        p = cls(fusion)

        def dev(a, dtype):
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(a)
            return t.to(device=device, dtype=dtype).contiguous()

        for op in spec:
            k = op[0]
            if k == "input":
                p.input(op[1])
            elif k == "const":
                p.const(dev(op[1], torch.float64))
            elif k == "scale":
                p.scale(op[1], op[2])
            elif k == "stencil":
                p.stencil(op[1], op[2], op[3])
            elif k == "gather":
                p.gather(op[1], dev(op[2], torch.int32), dev(op[3], torch.float64))
            elif k == "add":
                p.add(op[1], op[3], op[2], op[4])
            elif k == "mul":
                p.mul(op[1], op[2])
            elif k == "map":
                p.map(op[1], op[2])
            elif k == "scan":
                p.scan(op[1])
            elif k == "segsum":
                p.segment_sum(op[1], dev(op[2], torch.int64))
            elif k == "bcast":
                p.broadcast(op[1], dev(op[2], torch.int64), int(op[2][-1]))
            elif k == "sum":
                p.sum(op[1])
            else:
                raise PgError(EINVAL, "from_spec", f"unknown construct {k!r}")
        return p

    def _view(self, fn, where, *args) -> int:
        v = _I32()
        check(fn(self._p, *args, ctypes.byref(v)), where)
        return v.value

    def input(self, n: int) -> int:
        v = self._view(lib().pg_prog_input, "pg_prog_input", int(n))
        self.n_inputs += 1
        self.input_lengths.append(int(n))
        return v

    def const(self, data: torch.Tensor) -> int:
        _need_cuda(data)
        if data.dtype != torch.float64 or data.dim() != 1:
            raise PgError(EDTYPE, "const", "constants are 1-D float64 tensors")
        self._keep.append(data)
        return self._view(lib().pg_prog_const, "pg_prog_const", data.numel(), _ptr(data))

    def scale(self, a: int, alpha: float) -> int:
        return self._view(lib().pg_prog_scale, "pg_prog_scale", int(a), float(alpha))

    def stencil(self, a: int, offsets: Sequence[int], coeffs: Sequence[float]) -> int:
        n = len(offsets)
        if len(coeffs) != n:
            raise PgError(EINVAL, "stencil", "offsets and coeffs differ in length")
        off = (_I32 * max(n, 1))(*[int(o) for o in offsets])
        cf = (ctypes.c_double * max(n, 1))(*[float(c) for c in coeffs])
        return self._view(lib().pg_prog_stencil, "pg_prog_stencil", int(a), n, off, cf)

    def gather(self, a: int, conn: torch.Tensor, B: torch.Tensor) -> int:
        _need_cuda(conn, B)
        if conn.dtype != torch.int32 or B.dtype != torch.float64 or conn.dim() != 2 \
                or tuple(B.shape) != tuple(conn.shape):
            raise PgError(EDTYPE, "gather", "conn: (E, k) int32, B: (E, k) float64")
        self._keep += [conn, B]
        return self._view(lib().pg_prog_gather, "pg_prog_gather", int(a), conn.shape[0],
                          conn.shape[1], _ptr(conn), _ptr(B))

    def add(self, a: int, b: int, alpha: float = 1.0, beta: float = 1.0) -> int:
        return self._view(lib().pg_prog_add, "pg_prog_add", int(a), float(alpha), int(b),
                          float(beta))

    def mul(self, a: int, b: int) -> int:
        return self._view(lib().pg_prog_mul, "pg_prog_mul", int(a), int(b))

    def map(self, a: int, fn: str) -> int:
        return self._view(lib().pg_prog_map, "pg_prog_map", int(a), MAPS[fn])

    def scan(self, a: int) -> int:
        return self._view(lib().pg_prog_scan, "pg_prog_scan", int(a))

    def segment_sum(self, a: int, offsets: torch.Tensor) -> int:
        """y_s = sum of view a over [offsets[s], offsets[s+1]) (int64 offsets)."""
        _need_cuda(offsets)
        if offsets.dtype != torch.int64 or offsets.dim() != 1 or offsets.numel() < 1:
            raise PgError(EDTYPE, "segment_sum", "offsets: 1-D int64 with n_seg + 1 entries")
        self._keep.append(offsets)
        return self._view(lib().pg_prog_segment_sum, "pg_prog_segment_sum", int(a),
                          offsets.numel() - 1, _ptr(offsets))

    def broadcast(self, a: int, offsets: torch.Tensor, n_out: Optional[int] = None) -> int:
        """y_i = a_s for offsets[s] <= i < offsets[s+1]; n_out = offsets[-1]
        (read from the device when not given)."""
        _need_cuda(offsets)
        if offsets.dtype != torch.int64 or offsets.dim() != 1 or offsets.numel() < 1:
            raise PgError(EDTYPE, "broadcast", "offsets: 1-D int64 with len(a) + 1 entries")
        if n_out is None:
            n_out = int(offsets[-1].item())
        self._keep.append(offsets)
        return self._view(lib().pg_prog_broadcast, "pg_prog_broadcast", int(a), _ptr(offsets),
                          int(n_out))

    def sum(self, a: int) -> None:
        check(lib().pg_prog_sum(self._p, int(a)), "pg_prog_sum")

    def plan(self, device="cuda") -> "Program":
        sz = ctypes.c_size_t()
        check(lib().pg_prog_plan(self._p, ctypes.byref(sz)), "pg_prog_plan")
        self.workspace_bytes = sz.value
        raw = torch.empty(sz.value + WORKSPACE_ALIGN, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % WORKSPACE_ALIGN
        self._ws_raw = raw
        self._ws = raw[off:off + sz.value]
        torch.cuda.synchronize(device)  # operands are complete before the connectivity check
        check(lib().pg_prog_bind_workspace(self._p, ctypes.c_void_p(self._ws.data_ptr()),
                                           sz.value), "pg_prog_bind_workspace")
        return self

    def info(self) -> dict:
        st = ProgStats()
        check(lib().pg_prog_info(self._p, ctypes.byref(st)), "pg_prog_info")
        return {name: getattr(st, name) for name, _ in ProgStats._fields_}

    def run(self, inputs: Sequence[torch.Tensor], grads=True, stream=None, f_out=None,
            fbar: Optional[torch.Tensor] = None):
        """f (0-d float64 tensor) and, when grads is True (or a list of output
        tensors / None entries), the gradients with respect to the inputs,
        scaled by the device seed fbar (one float64; None means 1)."""
        if len(inputs) != self.n_inputs:
            raise PgError(EINVAL, "run", f"expected {self.n_inputs} inputs")
        for x, n in zip(inputs, self.input_lengths):
            _need_cuda(x)
            if x.dtype != torch.float64 or x.numel() != n:
                raise PgError(EDTYPE, "run", "inputs are float64 tensors of the declared lengths")
        dev = inputs[0].device if inputs else torch.device("cuda")
        f = torch.empty((), dtype=torch.float64, device=dev) if f_out is None else f_out
        ins = (_VP * max(self.n_inputs, 1))(*[x.data_ptr() for x in inputs])
        outs = None
        if grads is True:
            outs = [torch.empty_like(x) for x in inputs]
        elif grads:
            outs = list(grads)
            _need_cuda(*outs)
        gp = None
        if outs is not None:
            gp = (_VP * max(self.n_inputs, 1))(*[None if g is None else g.data_ptr() for g in outs])
        if fbar is not None:
            _need_cuda(fbar)
            if fbar.dtype != torch.float64 or fbar.numel() != 1:
                raise PgError(EDTYPE, "run", "fbar: one float64 on the device")
        check(lib().pg_prog_run(self._p, ins, _ptr(f), gp, _ptr(fbar), _stream(stream)),
              "pg_prog_run")
        return (f, outs) if outs is not None else f

    def close(self):
        if self._p:
            lib().pg_prog_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ autograd

def scale(alpha: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None,
          stream=None) -> torch.Tensor:
    """out = alpha[0] * x on the device (pg_scale; alpha one float64)."""
    _need_cuda(alpha, x, out)
    y = torch.empty_like(x) if out is None else out
    check(lib().pg_scale(_dtype_code(x), x.numel(), _ptr(alpha), _ptr(x), _ptr(y),
                         _stream(stream)), "pg_scale")
    return y


def mesh_gradient_noalloc(conn: torch.Tensor, B: torch.Tensor, w: torch.Tensor, x: torch.Tensor,
                          grad: torch.Tensor, f_out: torch.Tensor, stream=None) -> None:
    """pg_mesh_gradient_noalloc: the FP64 mesh gradient into caller-given grad
    (n_nodes) and f_out (one float64), with no plan, no workspace and no
    allocation (the library keeps the partial sums of f in a fixed device
    array).  conn: (n_elems, k) int32 with entries in [0, n_nodes), which
    this call does not check."""
    _need_cuda(conn, B, w, x, grad, f_out)
    n_elems, k = (conn.shape[0], conn.shape[1]) if conn.dim() == 2 else (conn.numel(), 1)
    check(lib().pg_mesh_gradient_noalloc(x.numel(), n_elems, k, _ptr(conn), _ptr(B), _ptr(w),
                                         _ptr(x), _ptr(grad), _ptr(f_out), _stream(stream)),
          "pg_mesh_gradient_noalloc")


def _seed(gout) -> torch.Tensor:
    if gout.dtype == torch.float64 and gout.is_contiguous():
        return gout.detach().reshape(-1)
    return gout.detach().to(torch.float64).contiguous().reshape(-1)


class _ObjectiveFn(torch.autograd.Function):
    """Shared forward/backward of the scalar-objective Functions.  The
    forward follows the objective's autograd_policy when a gradient will be
    needed (grad mode on and x requiring grad), and evaluates f alone
    otherwise."""

    @classmethod
    def apply(cls, x, obj):
        return super().apply(x, obj, bool(torch.is_grad_enabled() and x.requires_grad))

    @staticmethod
    def forward(ctx, x, obj, want_grad):
        xd = x.detach().contiguous()
        ctx.obj = obj
        ctx.policy = obj.autograd_policy if want_grad else "none"
        if ctx.policy == "gradient":
            f, g = obj.gradient(xd)
            ctx.save_for_backward(g)
        elif ctx.policy == "store":
            tape = obj.new_tape(xd.device)
            f = obj.objective_tape(xd, tape, f_shape=_ObjectiveFn._fshape(obj))
            ctx.save_for_backward(tape, xd)
        else:
            f = obj.objective(xd)
            ctx.save_for_backward(xd)
        return f

    @staticmethod
    def _fshape(obj):
        return (obj.n_inst,) if isinstance(obj, MeshBatch) else ()

    @staticmethod
    def backward(ctx, gout):
        fbar = _seed(gout)
        if ctx.policy == "gradient":
            (g,) = ctx.saved_tensors
            return scale(fbar, g), None, None
        if ctx.policy == "store":
            tape, xd = ctx.saved_tensors
            return ctx.obj.adjoint_tape(fbar, tape, xd), None, None
        if ctx.policy == "none":
            raise PgError(ESTATE, "backward", "the forward ran without a gradient requested")
        (xd,) = ctx.saved_tensors
        if ctx.obj._stores_tape():
            # A PG_STORE plan's adjoint reads the forward values its last
            # objective call kept in the workspace, which another forward may
            # have replaced since: record them again for this x first.
            ctx.obj._objective(xd, _ObjectiveFn._fshape(ctx.obj))
        return ctx.obj.adjoint(xd, fbar), None, None


class MeshFn(_ObjectiveFn):
    """y = f(x) for a MeshObjective.  What the forward keeps for the backward
    is the objective's autograd_policy: the gradient itself (f and the
    gradient in one pass; the backward multiplies by grad_output), u_e on a
    tape owned by this call, or nothing (the backward gathers x again)."""


class DenseFn(_ObjectiveFn):
    """y = f(x) for a DenseObjective (policies "gradient" or "recompute")."""


class BatchedDenseFn(_ObjectiveFn):
    """f(X) = sum W (.) psi(A X): forward product with the psi epilogue;
    the policy keeps the gradient, V = W (.) psi'(A X) on a per-call tape, or
    nothing (the backward recomputes V)."""


class MeshBatchFn(_ObjectiveFn):
    """Per-instance objectives of a MeshBatch (a vector output): the policy
    keeps u_e on a per-call tape or nothing; the backward seeds each
    instance with its own grad_output entry."""


class ProgramFn(torch.autograd.Function):
    """f = ProgramFn.apply(program, *inputs) for a planned Program; the
    backward runs the program's generated reverse pass seeded with
    grad_output (its forward values are recomputed there, as the fused
    groups do anyway)."""

    @staticmethod
    def forward(ctx, program: "Program", *inputs):
        xs = [x.detach().contiguous() for x in inputs]
        f = program.run(xs, grads=None)
        ctx.program = program
        ctx.save_for_backward(*xs)
        return f

    @staticmethod
    def backward(ctx, gout):
        xs = ctx.saved_tensors
        fbar = gout.detach().to(torch.float64).contiguous().reshape(1)
        want = [ctx.needs_input_grad[1 + i] for i in range(len(xs))]
        outs = [torch.empty_like(x) if w else None for x, w in zip(xs, want)]
        _, gs = ctx.program.run(list(xs), grads=outs, fbar=fbar)
        return (None, *gs)


