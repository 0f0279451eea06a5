"""Seeded synthetic inputs for every workload of the gradient library.

This module only draws random numbers and lays out index structures; it holds
none of the objective's arithmetic, so both the FP64 oracle and the HIP path
can take their inputs from it without sharing any of the method.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws its
arrays in a fixed order, so a (workload, seed) pair names one exact input.

Workloads (the paper's own example, section 4, is a 1D stencil on a vector of
up to 10,000 entries; the element form below generalises it):

* ``chain(n)``          -- 1D chain of n nodes, n-1 two-node elements,
                           B[e] = (-n, +n), w_e = 1/n, x ~ U(-1, 1)          (seed 0)
* ``hex_mesh(s)``       -- structured s^3 hex mesh, (s-1)^3 eight-node elements
                           in lexicographic order, B ~ N(0,1), w ~ U(0.5,1.5),
                           x ~ U(-1, 1)                                       (seed 1)
* ``dense(n)``          -- A n x n with entries N(0, 1/n), x ~ U(-1,1),
                           w ~ U(0.5,1.5)                                     (seed 2)
* ``batched_dense(m,n)``-- A m x m N(0, 1/m), X m x n ~ U(-1,1),
                           W m x n ~ U(0.5,1.5)                               (seed 3)
* ``uneven_batch(k)``   -- k hex meshes with side s = round(10**(1+U)),
                           U ~ U[0,1), concatenated                           (seed 4)
* ``ring_mesh(E, k)``   -- E elements on a ring of E nodes, element e on nodes
                           e, e+1, ..., e+k-1 (mod E): the largest incidence
                           count the int32 index range admits is E k < 2^31
* ``wide_index_mesh``   -- few elements on nodes at both ends of [0, 2^31 - 1),
                           x nonzero only on the nodes they touch
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_CHAIN = 0
SEED_HEX = 1
SEED_DENSE = 2
SEED_BDENSE = 3
SEED_BATCH = 4


@dataclasses.dataclass
class Mesh:
    """Element-connectivity workload: conn[E*k] int32, B[E*k], w[E], x[N]."""

    n_nodes: int
    n_elems: int
    k: int
    conn: np.ndarray  # int32, shape (E, k), row-major
    B: np.ndarray     # float64, shape (E, k)
    w: np.ndarray     # float64, shape (E,)
    x: np.ndarray     # float64, shape (N,)
    name: str = ""

    def astype(self, dtype) -> "Mesh":
        """Same mesh with B, w, x rounded to ``dtype`` (conn unchanged)."""
        return Mesh(self.n_nodes, self.n_elems, self.k, self.conn,
                    self.B.astype(dtype), self.w.astype(dtype),
                    self.x.astype(dtype), self.name)

    @property
    def nbytes_inputs(self) -> int:
        return self.conn.nbytes + self.B.nbytes + self.w.nbytes + self.x.nbytes


def chain_conn(n: int) -> np.ndarray:
    """Two-node elements (e, e+1) for e < n-1."""
    e = np.arange(max(n - 1, 0), dtype=np.int64)
    return np.stack([e, e + 1], axis=1).astype(np.int32)


def chain(n: int = 10_000, seed: int = SEED_CHAIN) -> Mesh:
    """1D chain: n nodes, E = n-1 elements, u_e = n (x_{e+1} - x_e), w_e = 1/n."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, n)
    E = max(n - 1, 0)
    conn = chain_conn(n)
    B = np.empty((E, 2), dtype=np.float64)
    B[:, 0] = -float(n)
    B[:, 1] = float(n)
    w = np.full(E, 1.0 / n, dtype=np.float64)
    return Mesh(n, E, 2, conn, B, w, x, f"chain{n}")


def hex_conn(s: int) -> np.ndarray:
    """Lexicographic connectivity of an s^3-node structured hex mesh.

    node(i, j, k) = i + s*(j + s*k), i fastest; element (i, j, k) with
    i, j, k < s-1 is numbered i + (s-1)*(j + (s-1)*k); its corner
    c = di + 2*dj + 4*dk is node(i+di, j+dj, k+dk).
    """
    m = s - 1
    if m <= 0:
        return np.zeros((0, 8), dtype=np.int32)
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    base = (ii + s * (jj + s * kk)).reshape(-1).astype(np.int64)
    conn = np.empty((base.size, 8), dtype=np.int64)
    for c in range(8):
        di, dj, dk = c & 1, (c >> 1) & 1, (c >> 2) & 1
        conn[:, c] = base + di + s * (dj + s * dk)
    return conn.astype(np.int32)


def hex_mesh(s: int = 128, seed: int = SEED_HEX, rng: Optional[np.random.Generator] = None) -> Mesh:
    """Structured hex mesh: x, then B, then w are drawn from one generator."""
    if rng is None:
        rng = np.random.default_rng(seed)
    N = s ** 3
    E = max(s - 1, 0) ** 3
    x = rng.uniform(-1.0, 1.0, N)
    B = rng.standard_normal((E, 8))
    w = rng.uniform(0.5, 1.5, E)
    return Mesh(N, E, 8, hex_conn(s), B, w, x, f"hex{s}")


def random_mesh(n_nodes: int, n_elems: int, k: int, seed: int) -> Mesh:
    """Unstructured mesh with uniformly random connectivity (repeats allowed)."""
    rng = np.random.default_rng(seed)
    conn = rng.integers(0, max(n_nodes, 1), size=(n_elems, k)).astype(np.int32)
    x = rng.uniform(-1.0, 1.0, n_nodes)
    B = rng.standard_normal((n_elems, k))
    w = rng.uniform(0.5, 1.5, n_elems)
    return Mesh(n_nodes, n_elems, k, conn, B, w, x, f"rand{n_nodes}x{n_elems}x{k}")


def ring_mesh(n_elems: int, k: int, seed: int = 7) -> Mesh:
    """E elements on a ring of E nodes, conn[e, j] = (e + j) mod E; B ~ N(0,1),
    w ~ U(0.5,1.5), x ~ U(-1,1) (drawn x, B, w).  Built in int32 without a
    64-bit intermediate so that E k close to 2^31 fits in host memory."""
    rng = np.random.default_rng(seed)
    E = n_elems
    conn = np.add.outer(np.arange(E, dtype=np.int32), np.arange(k, dtype=np.int32))
    conn[conn >= E] -= E
    x = rng.uniform(-1.0, 1.0, E)
    B = rng.standard_normal((E, k))
    w = rng.uniform(0.5, 1.5, E)
    return Mesh(E, E, k, conn, B, w, x, f"ring{E}x{k}")


@dataclasses.dataclass
class WideIndexMesh:
    """A mesh over n_nodes nodes whose x is zero except on the nodes the
    elements touch (x_nodes, ascending, with values x_vals)."""

    n_nodes: int
    n_elems: int
    k: int
    conn: np.ndarray
    B: np.ndarray
    w: np.ndarray
    x_nodes: np.ndarray  # int64, ascending
    x_vals: np.ndarray   # float64


def wide_index_mesh(n_nodes: int, n_elems: int, k: int, span: int, seed: int = 8) -> WideIndexMesh:
    """Connectivity uniform over [0, span) and [n_nodes - span, n_nodes) (half
    the incidences each, the last node always present), B ~ N(0,1),
    w ~ U(0.5,1.5), x ~ U(-1,1) on the touched nodes (drawn in this order:
    conn, B, w, x)."""
    rng = np.random.default_rng(seed)
    low = rng.integers(0, span, size=(n_elems, k))
    high = rng.integers(n_nodes - span, n_nodes, size=(n_elems, k))
    conn = np.where(rng.random((n_elems, k)) < 0.5, low, high)
    conn[-1, -1] = n_nodes - 1
    conn = conn.astype(np.int32)
    B = rng.standard_normal((n_elems, k))
    w = rng.uniform(0.5, 1.5, n_elems)
    nodes = np.unique(conn.astype(np.int64))
    x = rng.uniform(-1.0, 1.0, nodes.size)
    return WideIndexMesh(n_nodes, n_elems, k, conn, B, w, nodes, x)


@dataclasses.dataclass
class Dense:
    A: np.ndarray  # (rows, cols) float64 row-major
    x: np.ndarray  # (cols,)
    w: np.ndarray  # (rows,)


def dense(n: int = 10_000, seed: int = SEED_DENSE, rows: Optional[int] = None) -> Dense:
    """A ~ N(0, 1/cols), then x ~ U(-1,1), then w ~ U(0.5,1.5)."""
    rows = n if rows is None else rows
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((rows, n)) * (1.0 / np.sqrt(n))
    x = rng.uniform(-1.0, 1.0, n)
    w = rng.uniform(0.5, 1.5, rows)
    return Dense(A, x, w)


@dataclasses.dataclass
class BatchedDense:
    A: np.ndarray  # (m, m)
    X: np.ndarray  # (m, n)
    W: np.ndarray  # (m, n)


def batched_dense(m: int = 4096, n: int = 1024, seed: int = SEED_BDENSE) -> BatchedDense:
    """A ~ N(0, 1/m), then X ~ U(-1,1), then W ~ U(0.5,1.5)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, m)) * (1.0 / np.sqrt(m))
    X = rng.uniform(-1.0, 1.0, (m, n))
    W = rng.uniform(0.5, 1.5, (m, n))
    return BatchedDense(A, X, W)


def fd_directions(shape, count: int = 16, seed: int = 33) -> np.ndarray:
    """Random unit-norm directions for finite-difference checks."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count,) + tuple(shape))
    norms = np.sqrt((d.reshape(count, -1) ** 2).sum(axis=1))
    return d / norms.reshape((count,) + (1,) * len(shape))


@dataclasses.dataclass
class MeshBatch:
    """Concatenated meshes. inst[i] = (n_nodes, n_elems, node_off, elem_off).

    conn holds instance-local node numbers (0 <= conn < n_nodes of that
    instance); B, w are concatenated over elements, x over nodes.
    """

    inst: np.ndarray  # int64 (n_inst, 4)
    k: int
    conn: np.ndarray  # int32 (E_total, k)
    B: np.ndarray     # (E_total, k)
    w: np.ndarray     # (E_total,)
    x: np.ndarray     # (N_total,)
    sides: np.ndarray

    @property
    def n_inst(self) -> int:
        return int(self.inst.shape[0])

    def instance(self, i: int) -> Mesh:
        nn, ne, no, eo = (int(v) for v in self.inst[i])
        return Mesh(nn, ne, self.k, self.conn[eo:eo + ne], self.B[eo:eo + ne],
                    self.w[eo:eo + ne], self.x[no:no + nn], f"inst{i}")

    def astype(self, dtype) -> "MeshBatch":
        return MeshBatch(self.inst, self.k, self.conn, self.B.astype(dtype),
                         self.w.astype(dtype), self.x.astype(dtype), self.sides)


def uneven_sides(n_inst: int, seed: int = SEED_BATCH, lo: int = 10, hi: int = 100) -> np.ndarray:
    """Side lengths log-uniform in [lo, hi]: s = round(lo * (hi/lo)**U)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, n_inst)
    s = np.rint(lo * (hi / lo) ** u).astype(np.int64)
    return s, rng


def uneven_batch(n_inst: int = 256, seed: int = SEED_BATCH, lo: int = 10, hi: int = 100,
                 sides: Optional[List[int]] = None) -> MeshBatch:
    """Draw the sides, then for each instance x, B, w (same laws as hex_mesh)."""
    s_arr, rng = uneven_sides(n_inst, seed, lo, hi)
    if sides is not None:
        s_arr = np.asarray(sides, dtype=np.int64)
    conns, Bs, ws, xs = [], [], [], []
    inst = np.zeros((len(s_arr), 4), dtype=np.int64)
    no = eo = 0
    for i, s in enumerate(s_arr):
        m = hex_mesh(int(s), rng=rng)
        inst[i] = (m.n_nodes, m.n_elems, no, eo)
        no += m.n_nodes
        eo += m.n_elems
        conns.append(m.conn)
        Bs.append(m.B)
        ws.append(m.w)
        xs.append(m.x)
    conn = np.concatenate(conns) if conns else np.zeros((0, 8), np.int32)
    B = np.concatenate(Bs) if Bs else np.zeros((0, 8))
    w = np.concatenate(ws) if ws else np.zeros(0)
    x = np.concatenate(xs) if xs else np.zeros(0)
    return MeshBatch(inst, 8, conn, B, w, x, s_arr)


# ---------------------------------------------------------- composed programs
#
# A program is a list of constructs (tuples, view id = position in the list):
# ("input", n), ("const", data), ("scale", a, alpha), ("stencil", a, offsets,
# coeffs), ("gather", a, conn, B), ("add", a, alpha, b, beta), ("mul", a, b),
# ("map", a, "square" | "psi"), ("scan", a), and last ("sum", a).

@dataclasses.dataclass
class ProgramCase:
    spec: list
    inputs: List[np.ndarray]
    name: str


def program_mesh(m: Mesh) -> ProgramCase:
    """The element objective written as constructs: gather, map psi, weight, sum."""
    spec = [("input", m.n_nodes), ("gather", 0, m.conn, m.B), ("map", 1, "psi"),
            ("const", m.w), ("mul", 2, 3), ("sum", 4)]
    return ProgramCase(spec, [m.x], "mesh-" + m.name)


def program_paper(n: int, seed: int = SEED_CHAIN) -> ProgramCase:
    """The section 4 example as constructs: scale by 3, the Dirichlet 1D
    Laplacian stencil (-1, 2, -1), subtract b, square, sum; inputs x then b,
    both ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, n)
    b = rng.uniform(-1.0, 1.0, n)
    spec = [("input", n), ("input", n), ("scale", 0, 3.0),
            ("stencil", 2, [-1, 0, 1], [-1.0, 2.0, -1.0]), ("add", 3, 1.0, 1, -1.0),
            ("map", 4, "square"), ("sum", 5)]
    return ProgramCase(spec, [x, b], f"paper{n}")


def program_mix(n: int, n_elems: int, k: int, seed: int = 5, hot: int = 0) -> ProgramCase:
    """Every construct at least once, with active and inactive branches, two
    inputs, a self product and a gather whose reverse races.  hot > 0 draws
    the gather's connectivity from only the first `hot` entries (many
    colliding writes in the reverse pass)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, n)
    y = rng.uniform(-1.0, 1.0, n)
    c = rng.uniform(-1.0, 1.0, n)
    offs = [-2, -1, 0, 1, 3]
    coef = list(rng.uniform(-0.6, 0.6, len(offs)))
    top = hot if hot > 0 else max(n, 1)
    conn = rng.integers(0, top, size=(n_elems, k)).astype(np.int32)
    B = rng.standard_normal((n_elems, k)) / np.sqrt(k)
    wE = rng.uniform(0.5, 1.5, n_elems)
    spec = [
        ("input", n),                        # 0 x
        ("input", n),                        # 1 y
        ("const", c),                        # 2 c (inactive)
        ("stencil", 0, offs, coef),          # 3 active stencil: rescheduled reverse
        ("scale", 1, -0.7),                  # 4
        ("mul", 3, 4),                       # 5 both operands active
        ("add", 5, 0.3, 2, 1.1),             # 6 one operand inactive
        ("map", 6, "psi"),                   # 7
        ("scan", 7),                         # 8 prefix sum: reverse suffix scan
        ("scale", 8, 1.0 / max(n, 1)),       # 9
        ("stencil", 2, [0, 1], [1.0, -1.0]), # 10 inactive stencil: no reverse
        ("add", 9, 1.0, 10, 0.5),            # 11
        ("gather", 11, conn, B),             # 12 gather: atomic reverse
        ("mul", 12, 12),                     # 13 self product
        ("map", 12, "square"),               # 14
        ("add", 13, 0.25, 14, 0.75),         # 15
        ("const", wE),                       # 16
        ("mul", 15, 16),                     # 17
        ("sum", 17),
    ]
    return ProgramCase(spec, [x, y], f"mix{n}x{n_elems}x{k}" + (f"hot{hot}" if hot else ""))


def segment_offsets(n_seg: int, mean_len: float, seed: int, empty_frac: float = 0.1,
                    long_every: int = 97) -> np.ndarray:
    """Segment offsets (int64, n_seg + 1 entries): lengths ~ Poisson(mean_len),
    about `empty_frac` of the segments empty (and the middle one always),
    every `long_every`-th segment ten times longer (so one wave loops
    several times)."""
    rng = np.random.default_rng(seed)
    lens = rng.poisson(mean_len, n_seg)
    lens[rng.uniform(size=n_seg) < empty_frac] = 0
    lens[::long_every] *= 10
    if n_seg >= 3:
        lens[n_seg // 2] = 0  # at least one empty segment
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def program_segments(n_seg: int = 1000, mean_len: float = 20.0, seed: int = 6) -> ProgramCase:
    """Segment sums and broadcasts with active and inactive operands:
    f = sum(x * bcast(psi(segsum(x)))) + sum(scale(segsum(x * c)))."""
    off = segment_offsets(n_seg, mean_len, seed)
    n = int(off[-1])
    rng = np.random.default_rng(seed + 1)
    x = rng.uniform(-1.0, 1.0, n)
    c = rng.uniform(-1.0, 1.0, n)
    spec = [
        ("input", n),              # 0 x
        ("segsum", 0, off),        # 1 per-segment sums
        ("map", 1, "psi"),         # 2
        ("bcast", 2, off),         # 3 back to entries
        ("mul", 3, 0),             # 4
        ("const", c),              # 5
        ("mul", 0, 5),             # 6
        ("segsum", 6, off),        # 7
        ("scale", 7, 0.5),         # 8
        ("bcast", 8, off),         # 9
        ("add", 4, 1.0, 9, 1.0),   # 10
        ("sum", 10),
    ]
    return ProgramCase(spec, [x], f"segments{n_seg}")
