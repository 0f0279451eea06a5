"""FP64 CPU oracle for the reverse-mode gradient library (ctypes over oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path never does.
It shares no code with the HIP path (see oracle.c for what it computes and
which part of the paper each step follows).

Batched dense: the fast form uses NumPy's FP64 matrix product as a library
primitive for A @ X and A.T @ V; the accurate form (Dot2 per column, in C) is
used on selected columns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ERANGE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FP contraction) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_omp = None
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build_omp(force: bool = True) -> str:
    """The same source built with OpenMP (-DORC_OMP): adds the threaded mesh
    gradient used to time the oracle on every host core."""
    if force or not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
        tmp = _LIB_OMP + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-fopenmp",
                               "-DORC_OMP", "-std=c11", "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_OMP)
    return _LIB_OMP


def lib_omp():
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
            build_omp(force=True)
        L = ctypes.CDLL(_LIB_OMP)
        L.orc_mesh_gradient_threads.argtypes = [_I64, _I64, _I32, _i32, _d, _d, _d, ctypes.c_double,
                                                _d, _d]
        L.orc_mesh_gradient_threads.restype = ctypes.c_int
        _lib_omp = L
    return _lib_omp

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        for name in ("orc_psi", "orc_dpsi", "orc_ddpsi"):
            getattr(L, name).argtypes = [_I64, _d, _d]
            getattr(L, name).restype = ctypes.c_int
        L.orc_mesh_check.argtypes = [_I64, _I64, _I32, _i32]
        L.orc_mesh_gather.argtypes = [_I64, _I64, _I32, _i32, _d, _d, _d]
        L.orc_mesh_scatter.argtypes = [_I64, _I64, _I32, _i32, _d, _d, _d]
        L.orc_mesh_terms.argtypes = [_I64, _I64, _I32, _i32, _d, _d, _d, _d, _d]
        L.orc_mesh_objective.argtypes = [_I64, _I64, _I32, _i32, _d, _d, _d, _d]
        L.orc_mesh_gradient.argtypes = [_I64, _I64, _I32, _i32, _d, _d, _d, ctypes.c_double, _d, _d]
        L.orc_mesh_hvp.argtypes = [_I64, _I64, _I32, _i32, _d, _d, _d, _d, _d]
        L.orc_mesh_csr.argtypes = [_I64, _I64, _I32, _i32, _i32, _i32]
        L.orc_colour_conflicts.argtypes = [_I64, _I64, _I32, _i32, _i32, _I32]
        L.orc_colour_conflicts.restype = ctypes.c_int64
        L.orc_greedy_colour.argtypes = [_I64, _I64, _I32, _i32, _I32, _i32]
        L.orc_greedy_colour.restype = ctypes.c_int32
        L.orc_dense_objective.argtypes = [_I64, _I64, _d, _d, _d, _d, _d]
        L.orc_dense_gradient.argtypes = [_I64, _I64, _d, _d, _d, ctypes.c_double, _d, _d]
        L.orc_bdense_columns.argtypes = [_I64, _I64, _d, _d, _d, _I64, _i64p, _d, _d]
        L.orc_laplace1d_gradient.argtypes = [_I64, _d, _d, ctypes.c_double, _d, _d, _d]
        L.orc_laplace1d_gradient.restype = ctypes.c_int
        L.orc_sum.argtypes = [_I64, _d]
        L.orc_sum.restype = ctypes.c_double
        for name in ("orc_mesh_check", "orc_mesh_gather", "orc_mesh_scatter", "orc_mesh_terms",
                     "orc_mesh_objective", "orc_mesh_gradient", "orc_mesh_hvp", "orc_mesh_csr",
                     "orc_dense_objective", "orc_dense_gradient", "orc_bdense_columns"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what}: status {code}")
        self.code = code


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32a(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a: Optional[np.ndarray], t=_d):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _chk(code: int, what: str):
    if code != OK:
        raise OracleError(code, what)


# ------------------------------------------------------------------ scalars

def psi(s) -> np.ndarray:
    s = _f64(np.atleast_1d(s))
    out = np.empty_like(s)
    _chk(lib().orc_psi(s.size, _p(s), _p(out)), "psi")
    return out


def dpsi(s) -> np.ndarray:
    s = _f64(np.atleast_1d(s))
    out = np.empty_like(s)
    _chk(lib().orc_dpsi(s.size, _p(s), _p(out)), "dpsi")
    return out


def ddpsi(s) -> np.ndarray:
    s = _f64(np.atleast_1d(s))
    out = np.empty_like(s)
    _chk(lib().orc_ddpsi(s.size, _p(s), _p(out)), "ddpsi")
    return out


def fsum(a) -> float:
    a = _f64(a).ravel()
    return float(lib().orc_sum(a.size, _p(a)))


# ------------------------------------------------------------------- meshes

def _mesh_args(n_nodes, conn, B):
    conn = _i32a(conn)
    E = conn.shape[0] if conn.ndim == 2 else 0
    k = conn.shape[1] if conn.ndim == 2 else 1
    return int(n_nodes), E, k, conn, _f64(B)


def mesh_check(n_nodes, conn) -> int:
    conn = _i32a(conn)
    E, k = conn.shape
    return lib().orc_mesh_check(int(n_nodes), E, k, _p(conn, _i32))


def mesh_gather(n_nodes, conn, B, x) -> np.ndarray:
    N, E, k, conn, B = _mesh_args(n_nodes, conn, B)
    x = _f64(x)
    u = np.empty(E)
    _chk(lib().orc_mesh_gather(N, E, k, _p(conn, _i32), _p(B), _p(x), _p(u)), "gather")
    return u


def mesh_scatter(n_nodes, conn, B, v) -> np.ndarray:
    N, E, k, conn, B = _mesh_args(n_nodes, conn, B)
    v = _f64(v)
    g = np.empty(N)
    _chk(lib().orc_mesh_scatter(N, E, k, _p(conn, _i32), _p(B), _p(v), _p(g)), "scatter")
    return g


def mesh_terms(n_nodes, conn, B, w, x) -> Tuple[np.ndarray, np.ndarray]:
    N, E, k, conn, B = _mesh_args(n_nodes, conn, B)
    w, x = _f64(w), _f64(x)
    t = np.empty(E)
    u = np.empty(E)
    _chk(lib().orc_mesh_terms(N, E, k, _p(conn, _i32), _p(B), _p(w), _p(x), _p(t), _p(u)),
         "terms")
    return t, u


def mesh_objective(n_nodes, conn, B, w, x) -> float:
    N, E, k, conn, B = _mesh_args(n_nodes, conn, B)
    w, x = _f64(w), _f64(x)
    f = np.zeros(1)
    _chk(lib().orc_mesh_objective(N, E, k, _p(conn, _i32), _p(B), _p(w), _p(x), _p(f)),
         "objective")
    return float(f[0])


def mesh_gradient(n_nodes, conn, B, w, x, fbar: float = 1.0) -> Tuple[float, np.ndarray]:
    N, E, k, conn, B = _mesh_args(n_nodes, conn, B)
    w, x = _f64(w), _f64(x)
    f = np.zeros(1)
    g = np.empty(N)
    _chk(lib().orc_mesh_gradient(N, E, k, _p(conn, _i32), _p(B), _p(w), _p(x), float(fbar),
                                 _p(f), _p(g)), "gradient")
    return float(f[0]), g


def mesh_gradient_threads(n_nodes, conn, B, w, x, fbar: float = 1.0) -> Tuple[float, np.ndarray, int]:
    """mesh_gradient with its loops on every host thread (OpenMP build):
    (f, grad, threads used).  For timing the oracle on the host's cores."""
    N, E, k, conn, B = _mesh_args(n_nodes, conn, B)
    w, x = _f64(w), _f64(x)
    g = np.empty(N)
    f = ctypes.c_double()
    t = lib_omp().orc_mesh_gradient_threads(N, E, k, _p(conn, _i32), _p(B), _p(w), _p(x),
                                             float(fbar), ctypes.byref(f), _p(g))
    if t < 0:
        raise OracleError(-t, "mesh_gradient_threads")
    return f.value, g, int(t)


def mesh_hvp(n_nodes, conn, B, w, x, d) -> np.ndarray:
    N, E, k, conn, B = _mesh_args(n_nodes, conn, B)
    w, x, d = _f64(w), _f64(x), _f64(d)
    hd = np.empty(N)
    _chk(lib().orc_mesh_hvp(N, E, k, _p(conn, _i32), _p(B), _p(w), _p(x), _p(d), _p(hd)), "hvp")
    return hd


def mesh_csr(n_nodes, conn) -> Tuple[np.ndarray, np.ndarray]:
    conn = _i32a(conn)
    E, k = conn.shape
    offs = np.empty(int(n_nodes) + 1, dtype=np.int32)
    inc = np.empty(E * k, dtype=np.int32)
    _chk(lib().orc_mesh_csr(int(n_nodes), E, k, _p(conn, _i32), _p(offs, _i32), _p(inc, _i32)),
         "csr")
    return offs, inc


def greedy_colour(n_nodes, conn, max_colours: int = 64) -> Tuple[np.ndarray, int]:
    """Greedy colouring in element order (smallest colour no earlier element
    sharing a node has); returns (colour per element, number of colours)."""
    conn = _i32a(conn)
    E, k = conn.shape
    colour = np.zeros(E, dtype=np.int32)
    nc = int(lib().orc_greedy_colour(int(n_nodes), E, k, _p(conn, _i32), int(max_colours),
                                     _p(colour, _i32)))
    if nc < 0:
        raise OracleError(EINVAL, "greedy_colour")
    return colour, nc


def colour_conflicts(n_nodes, conn, colour, n_colours: int) -> int:
    conn = _i32a(conn)
    colour = _i32a(colour)
    E, k = conn.shape
    return int(lib().orc_colour_conflicts(int(n_nodes), E, k, _p(conn, _i32), _p(colour, _i32),
                                          int(n_colours)))


def mesh_batch_gradient(batch, fbar: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Per-instance f and the concatenated gradient of a MeshBatch."""
    fs = np.empty(batch.n_inst)
    g = np.empty(batch.x.shape[0])
    for i in range(batch.n_inst):
        m = batch.instance(i)
        nn, _, no, _ = (int(v) for v in batch.inst[i])
        fs[i], g[no:no + nn] = mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x, fbar)
    return fs, g


def mesh_batch_objective(batch) -> np.ndarray:
    fs = np.empty(batch.n_inst)
    for i in range(batch.n_inst):
        m = batch.instance(i)
        fs[i] = mesh_objective(m.n_nodes, m.conn, m.B, m.w, m.x)
    return fs


# -------------------------------------------------------------------- dense

def dense_objective(A, x, w) -> Tuple[float, np.ndarray]:
    A = _f64(A)
    rows, cols = A.shape
    x, w = _f64(x), _f64(w)
    f = np.zeros(1)
    r = np.empty(rows)
    _chk(lib().orc_dense_objective(rows, cols, _p(A), _p(x), _p(w), _p(f), _p(r)), "dense")
    return float(f[0]), r


def dense_gradient(A, x, w, fbar: float = 1.0) -> Tuple[float, np.ndarray]:
    A = _f64(A)
    rows, cols = A.shape
    x, w = _f64(x), _f64(w)
    f = np.zeros(1)
    g = np.empty(cols)
    _chk(lib().orc_dense_gradient(rows, cols, _p(A), _p(x), _p(w), float(fbar), _p(f), _p(g)),
         "dense grad")
    return float(f[0]), g


def bdense_columns(A, X, W, cols: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Accurate (Dot2) per-column objective and gradient columns."""
    A, X, W = _f64(A), _f64(X), _f64(W)
    m, n = X.shape
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    fc = np.empty(cols.size)
    G = np.empty((m, cols.size))
    _chk(lib().orc_bdense_columns(m, n, _p(A), _p(X), _p(W), cols.size, _p(cols, _i64p),
                                  _p(fc), _p(G)), "bdense")
    return fc, G


def bdense_gradient_fast(A, X, W, fbar: float = 1.0) -> Tuple[float, np.ndarray]:
    """f = sum W psi(A X), G = A^T (fbar W psi'(A X)); NumPy matmul as the
    contraction primitive, psi/psi' and the compensated sum from oracle.c."""
    A, X, W = _f64(A), _f64(X), _f64(W)
    Y = A @ X
    t = W * psi(Y.ravel()).reshape(Y.shape)
    f = fsum(t)
    V = fbar * W * dpsi(Y.ravel()).reshape(Y.shape)
    return f, A.T @ V


# ------------------------------------------- the paper's section 4 example

def laplace1d_gradient(x, b, fbar: float = 1.0):
    """f(x, b) = ||A(3x) - b||^2 (A: 1D Laplacian), and its gradients in x and b."""
    x, b = _f64(x), _f64(b)
    n = x.size
    f = np.zeros(1)
    gx = np.empty(n)
    gb = np.empty(n)
    _chk(lib().orc_laplace1d_gradient(n, _p(x), _p(b), float(fbar), _p(f), _p(gx), _p(gb)),
         "laplace1d")
    return float(f[0]), gx, gb
