"""Composed programs: values, and gradients by forward Jacobian accumulation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.

A program is a list of constructs, each producing one view from earlier views
(the data-parallel kernels of section 2, chained as in section 4, ending in a
parallel sum).  Constructs, as tuples:

    ("input", n)                        active input of n entries
    ("const", data)                     inactive operand
    ("scale", a, alpha)                 y = alpha a
    ("stencil", a, offsets, coeffs)     y_i = sum_t c_t a_{i+o_t}, taps outside [0, n) dropped
    ("gather", a, conn, B)              y_e = sum_j B[e, j] a[conn[e, j]]
    ("add", a, alpha, b, beta)          y = alpha a + beta b
    ("mul", a, b)                       y = a * b (elementwise)
    ("map", a, fn)                      y = fn(a): "square" (s^2) or "psi" (the element
                                        nonlinearity psi(s) = s^2/2 + log(1 + s^2)/2)
    ("scan", a)                         y_i = sum_{j <= i} a_j (inclusive prefix sum)
    ("segsum", a, offsets)              y_s = sum of a over [offsets[s], offsets[s+1])
    ("bcast", a, offsets)               y_i = a_s for offsets[s] <= i < offsets[s+1]
    ("sum", a)                          f = sum of view a; must come last

View ids are the positions of the constructs in the list.

The gradient is NOT computed by a reverse pass.  For every view the oracle
forms the explicit sparse Jacobian of that view with respect to every input,
in program order, by the chain rule (the derivative of a composition of the
kernels, section 2), with scipy.sparse matrices; the gradient of f = sum(v)
with respect to input i is then the vector of column sums of dv/dx_i.  No
adjoint statement, shadow accumulation, atomic or rescheduling appears, so the
result checks the reverse pass of section 3 from a different formulation.
Plain NumPy evaluates the values; complex inputs are accepted so that the
complex-step derivative can pin the Jacobians.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp


def _phi(fn: str, s):
    if fn == "square":
        return s * s
    if fn == "psi":
        return 0.5 * s * s + 0.5 * np.log1p(s * s)
    raise ValueError(f"unknown map {fn!r}")


def _dphi(fn: str, s):
    if fn == "square":
        return 2.0 * s
    if fn == "psi":
        return s + s / (1.0 + s * s)
    raise ValueError(f"unknown map {fn!r}")


def _stencil_matrix(n: int, offsets, coeffs) -> sp.csr_matrix:
    rows, cols, vals = [], [], []
    i = np.arange(n)
    for o, c in zip(offsets, coeffs):
        j = i + int(o)
        ok = (j >= 0) & (j < n)
        rows.append(i[ok])
        cols.append(j[ok])
        vals.append(np.full(int(ok.sum()), float(c)))
    if not rows:
        return sp.csr_matrix((n, n))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def _gather_matrix(n_in: int, conn, B) -> sp.csr_matrix:
    conn = np.asarray(conn).reshape(len(conn), -1)
    B = np.asarray(B, dtype=np.float64).reshape(conn.shape)
    E, k = conn.shape
    rows = np.repeat(np.arange(E), k)
    return sp.csr_matrix((B.ravel(), (rows, conn.ravel().astype(np.int64))), shape=(E, n_in))


def _scan_matrix(n: int) -> sp.csr_matrix:
    return sp.csr_matrix(np.tril(np.ones((n, n))))


def _segment_matrix(offsets) -> sp.csr_matrix:
    """S[s, i] = 1 for offsets[s] <= i < offsets[s+1]: the segment sum."""
    off = np.asarray(offsets, dtype=np.int64)
    n_seg, n = len(off) - 1, int(off[-1])
    rows = np.repeat(np.arange(n_seg), np.diff(off))
    return sp.csr_matrix((np.ones(n), (rows, np.arange(n))), shape=(n_seg, n))


def lengths(spec) -> List[int]:
    """Length of every view (the sum construct gets length 1)."""
    out: List[int] = []
    for op in spec:
        k = op[0]
        if k == "input":
            out.append(int(op[1]))
        elif k == "const":
            out.append(len(op[1]))
        elif k == "gather":
            out.append(len(op[2]))
        elif k == "segsum":
            out.append(len(op[2]) - 1)
        elif k == "bcast":
            out.append(int(op[2][-1]))
        elif k == "sum":
            out.append(1)
        else:
            out.append(out[op[1]])
    return out


def values(spec, inputs: Sequence[np.ndarray]) -> list:
    """Forward values of every view (the sum construct's entry is f)."""
    vals: list = []
    nin = 0
    for op in spec:
        k = op[0]
        if k == "input":
            vals.append(np.asarray(inputs[nin]))
            nin += 1
        elif k == "const":
            vals.append(np.asarray(op[1], dtype=np.float64))
        elif k == "scale":
            vals.append(op[2] * vals[op[1]])
        elif k == "stencil":
            a = vals[op[1]]
            vals.append(_stencil_matrix(len(a), op[2], op[3]) @ a)
        elif k == "gather":
            vals.append(_gather_matrix(len(vals[op[1]]), op[2], op[3]) @ vals[op[1]])
        elif k == "add":
            vals.append(op[2] * vals[op[1]] + op[4] * vals[op[3]])
        elif k == "mul":
            vals.append(vals[op[1]] * vals[op[2]])
        elif k == "map":
            vals.append(_phi(op[2], vals[op[1]]))
        elif k == "scan":
            vals.append(np.cumsum(vals[op[1]]))
        elif k == "segsum":
            vals.append(_segment_matrix(op[2]) @ vals[op[1]])
        elif k == "bcast":
            vals.append(_segment_matrix(op[2]).T @ vals[op[1]])
        elif k == "sum":
            v = vals[op[1]]
            vals.append(math.fsum(v) if np.isrealobj(v) else np.sum(v))
        else:
            raise ValueError(f"unknown construct {k!r}")
    return vals


def objective(spec, inputs: Sequence[np.ndarray]) -> float:
    """f, the last construct's value (correctly rounded sum of the summed view)."""
    return float(values(spec, [np.asarray(x, dtype=np.float64) for x in inputs])[-1])


def gradient(spec, inputs: Sequence[np.ndarray]) -> Tuple[float, List[np.ndarray]]:
    """f and df/d(input i) for every input, by forward Jacobian accumulation."""
    inputs = [np.asarray(x, dtype=np.float64) for x in inputs]
    vals = values(spec, inputs)
    n_in = [len(x) for x in inputs]
    jac: List[dict] = []   # jac[v][i]: sparse d(view v)/d(input i)
    nin = 0
    for v, op in enumerate(spec):
        k = op[0]
        J: dict = {}

        def acc(src: int, M):
            for i, Ji in jac[src].items():
                t = M @ Ji
                J[i] = J[i] + t if i in J else t

        if k == "input":
            J[nin] = sp.identity(n_in[nin], format="csr")
            nin += 1
        elif k == "const":
            pass
        elif k == "scale":
            acc(op[1], op[2] * sp.identity(len(vals[v]), format="csr"))
        elif k == "stencil":
            acc(op[1], _stencil_matrix(len(vals[v]), op[2], op[3]))
        elif k == "gather":
            acc(op[1], _gather_matrix(len(vals[op[1]]), op[2], op[3]))
        elif k == "add":
            acc(op[1], op[2] * sp.identity(len(vals[v]), format="csr"))
            acc(op[3], op[4] * sp.identity(len(vals[v]), format="csr"))
        elif k == "mul":
            acc(op[1], sp.diags(vals[op[2]], format="csr"))
            acc(op[2], sp.diags(vals[op[1]], format="csr"))
        elif k == "map":
            acc(op[1], sp.diags(_dphi(op[2], vals[op[1]]), format="csr"))
        elif k == "scan":
            acc(op[1], _scan_matrix(len(vals[v])))
        elif k == "segsum":
            acc(op[1], _segment_matrix(op[2]))
        elif k == "bcast":
            acc(op[1], _segment_matrix(op[2]).T.tocsr())
        elif k == "sum":
            acc(op[1], sp.csr_matrix(np.ones((1, len(vals[op[1]])))))
        jac.append(J)
    last = jac[-1]
    grads = []
    for i in range(len(inputs)):
        g = last[i].toarray().ravel() if i in last else np.zeros(n_in[i])
        grads.append(np.asarray(g, dtype=np.float64))
    return float(vals[-1]), grads


def complex_step(spec, inputs: Sequence[np.ndarray], which: int, j: int,
                 h: float = 1e-30) -> float:
    """df/d(input which)[j] by the complex step Im f(x + i h e_j) / h."""
    xs = [np.asarray(x, dtype=np.complex128).copy() for x in inputs]
    xs[which][j] += 1j * h
    return float(np.imag(values(spec, xs)[-1]) / h)


def sampled_gradient(spec, inputs: Sequence[np.ndarray], which: int,
                     idx: Sequence[int]) -> np.ndarray:
    """Selected entries of df/d(input which), one complex-step evaluation each
    (for sizes where the explicit Jacobians would not fit)."""
    return np.array([complex_step(spec, inputs, which, int(j)) for j in idx])
