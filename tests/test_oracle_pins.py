"""Pins of the FP64 oracle against what mathematics fixes (no GPU).

Each test ties the oracle to something other than itself: closed forms of
worked examples, a complex-step derivative written independently in pure
Python, exact rational arithmetic, SciPy / NumPy library routines, central
finite differences, the adjoint (dot-product) identity and metamorphic
relations.  A dropped term, a wrong sign, a wrong index or a transposed
operand anywhere in the oracle fails at least one of them.
"""
import cmath
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2507_13204_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "chain_worked.json")


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


# ------------------------------------------------------------ psi and psi'

def test_psi_closed_form_values(orc):
    g = json.load(open(GOLD))["psi_values"]
    s = np.array(g["s"])
    exact_psi = [0.0, 0.5 + math.log(2) / 2, 2 + math.log(5) / 2, 0.5 + math.log(2) / 2,
                 2 + math.log(5) / 2]
    assert np.allclose(g["psi"], exact_psi, rtol=0, atol=4e-16)
    p = orc.psi(s)
    d = orc.dpsi(s)
    for got, want in zip(p, g["psi"]):
        assert abs(got - want) <= 2 * np.spacing(max(abs(want), 1e-300))
    assert np.array_equal(d, np.array(g["dpsi"]))  # exact: 1.5, 2.4 are single roundings


def test_psi_symmetry_and_derivatives(orc):
    s = np.linspace(-7.0, 7.0, 1001)
    assert np.array_equal(orc.psi(s), orc.psi(-s))          # psi even
    assert np.array_equal(orc.dpsi(s), -orc.dpsi(-s))       # psi' odd
    # psi' is the derivative of psi: central differences (h^2 error)
    h = 1e-5
    fd = (orc.psi(s + h) - orc.psi(s - h)) / (2 * h)
    assert np.max(np.abs(fd - orc.dpsi(s)) / (1 + np.abs(s))) < 1e-8
    fd2 = (orc.dpsi(s + h) - orc.dpsi(s - h)) / (2 * h)
    assert np.max(np.abs(fd2 - orc.ddpsi(s))) < 1e-8
    dd = orc.ddpsi(s)
    assert dd.min() >= 7.0 / 8.0 - 1e-15 and dd.max() <= 2.0 + 1e-15  # psi'' in [7/8, 2]
    # small-argument series psi(s) = s^2 - s^4/4 + ..., psi'(s) = 2s - s^3 + ...
    t = np.array([1e-9, -3e-8, 2e-6])
    assert np.allclose(orc.psi(t), t * t - t ** 4 / 4, rtol=1e-12, atol=0)
    assert np.allclose(orc.dpsi(t), 2 * t - t ** 3, rtol=1e-12, atol=0)


# ------------------------------------------------------ worked 1D examples

@pytest.mark.parametrize("case", json.load(open(GOLD))["cases"], ids=lambda c: f"n{c['n']}")
def test_chain_worked_examples(orc, case):
    n = case["n"]
    m = inputs.chain(n)
    x = np.array(case["x"])
    u = orc.mesh_gather(m.n_nodes, m.conn, m.B, x)
    assert np.array_equal(u, np.array(case["u"]))
    f, g = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, x)
    assert abs(f - case["f"]) <= 1e-15 * abs(case["f"])
    assert np.allclose(g, case["g"], rtol=1e-15, atol=1e-15)


def test_chain_closed_form_full_size(orc):
    """1D chain, n = 10,000: g_i = [i>=1] psi'(u_{i-1}) - [i<=n-2] psi'(u_i)."""
    m = inputs.chain(10_000)
    f, g = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    u = m.n_nodes * (m.x[1:] - m.x[:-1])
    dp = u + u / (1 + u * u)
    want = np.zeros(m.n_nodes)
    want[1:] += dp
    want[:-1] -= dp
    assert rel(g, want) <= 1e-14
    # B rows sum to zero, so f is translation invariant and the gradient sums to 0
    assert abs(g.sum()) <= 1e-12 * np.abs(g).sum()
    f_shift = orc.mesh_objective(m.n_nodes, m.conn, m.B, m.w, m.x + 0.125)
    assert abs(f_shift - f) <= 1e-9 * abs(f)
    assert 1e6 < f < 1e9 and np.abs(g).max() > 1e3


# ------------------------------------------------ linear operator G and G^T

def _sparse_G(m):
    rows = np.repeat(np.arange(m.n_elems), m.k)
    return sp.csr_matrix((m.B.ravel(), (rows, m.conn.ravel().astype(np.int64))),
                         shape=(m.n_elems, m.n_nodes))  # duplicates add


@pytest.mark.parametrize("mesh", [inputs.hex_mesh(9, seed=11), inputs.random_mesh(300, 500, 5, 12),
                                  inputs.chain(77)], ids=["hex9", "rand", "chain"])
def test_gather_scatter_vs_scipy_and_adjoint(orc, mesh):
    G = _sparse_G(mesh)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(mesh.n_nodes)
    v = rng.standard_normal(mesh.n_elems)
    Gx = orc.mesh_gather(mesh.n_nodes, mesh.conn, mesh.B, x)
    Gtv = orc.mesh_scatter(mesh.n_nodes, mesh.conn, mesh.B, v)
    assert rel(Gx, G @ x) <= 1e-13
    assert rel(Gtv, G.T @ v) <= 1e-13
    lhs, rhs = float(Gx @ v), float(x @ Gtv)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Gx) * np.linalg.norm(v)


# ---------------------------------- complex-step derivative, brute force

def _cs_objective(n_nodes, conn, B, w, xc):
    """Pure-Python complex evaluation of f; independent of oracle.c."""
    total = 0j
    for e in range(conn.shape[0]):
        s = 0j
        for j in range(conn.shape[1]):
            s += float(B[e, j]) * xc[int(conn[e, j])]
        total += float(w[e]) * (0.5 * s * s + 0.5 * cmath.log(1 + s * s))
    return total


def _cs_gradient(mesh, x, h=1e-30):
    g = np.empty(mesh.n_nodes)
    base = [complex(v) for v in x]
    for i in range(mesh.n_nodes):
        xc = list(base)
        xc[i] = complex(x[i], h)
        g[i] = _cs_objective(mesh.n_nodes, mesh.conn, mesh.B, mesh.w, xc).imag / h
    return _cs_objective(mesh.n_nodes, mesh.conn, mesh.B, mesh.w, base).real, g


@pytest.mark.parametrize("mesh", [inputs.hex_mesh(3, seed=21), inputs.random_mesh(10, 7, 4, 22),
                                  inputs.random_mesh(5, 9, 3, 23), inputs.chain(6, seed=24)],
                         ids=["hex3", "rand10", "rand5_repeats", "chain6"])
def test_gradient_complex_step(orc, mesh):
    f, g = orc.mesh_gradient(mesh.n_nodes, mesh.conn, mesh.B, mesh.w, mesh.x)
    fc, gc = _cs_gradient(mesh, mesh.x)
    assert abs(f - fc) <= 1e-14 * abs(fc)
    assert rel(g, gc) <= 1e-14


def test_gradient_seed_scaling(orc):
    """The seed fbar multiplies the whole reverse pass (adjoint of the output)."""
    m = inputs.hex_mesh(6, seed=3)
    _, g1 = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x, 1.0)
    _, g3 = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x, -0.75)
    assert rel(g3, -0.75 * g1) <= 1e-15


# --------------------------------------------- finite differences / Taylor

def test_gradient_finite_differences_and_taylor(orc):
    m = inputs.hex_mesh(12, seed=31)
    f0, g = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    dirs = inputs.fd_directions((m.n_nodes,), 16, seed=33)
    F = lambda x: orc.mesh_objective(m.n_nodes, m.conn, m.B, m.w, x)
    for d in dirs:
        h = 1e-5
        fd = (F(m.x + h * d) - F(m.x - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(g @ d), np.linalg.norm(g) * 1e-3)
    d = dirs[0]
    hs = np.array([1e-1, 3e-2, 1e-2, 3e-3, 1e-3])
    r = np.array([abs(F(m.x + h * d) - f0 - h * (g @ d)) for h in hs])
    slope = np.polyfit(np.log(hs), np.log(r), 1)[0]
    assert 1.9 <= slope <= 2.1


def test_objective_fsum(orc):
    m = inputs.hex_mesh(20, seed=41)
    t, u = orc.mesh_terms(m.n_nodes, m.conn, m.B, m.w, m.x)
    f = orc.mesh_objective(m.n_nodes, m.conn, m.B, m.w, m.x)
    assert abs(f - math.fsum(t)) <= 1e-15 * abs(f)
    assert rel(u, _sparse_G(m) @ m.x) <= 1e-13


# ------------------------------------------------------------ metamorphic

def test_metamorphic_relations(orc):
    m = inputs.hex_mesh(7, seed=51)
    N = m.n_nodes
    f, g = orc.mesh_gradient(N, m.conn, m.B, m.w, m.x)
    # w -> 4w scales f and g exactly
    f4, g4 = orc.mesh_gradient(N, m.conn, m.B, 4.0 * m.w, m.x)
    assert f4 == 4.0 * f and np.array_equal(g4, 4.0 * g)
    # B -> -B leaves f and g unchanged (psi even, psi' odd)
    fn, gn = orc.mesh_gradient(N, m.conn, -m.B, m.w, m.x)
    assert fn == f and np.array_equal(gn, g)
    # relabel nodes by a permutation pi: g permuted the same way, exactly
    pi = np.random.default_rng(1).permutation(N)
    inv = np.argsort(pi)
    conn_p = inv[m.conn].astype(np.int32)
    x_p = m.x[pi]
    fp, gp = orc.mesh_gradient(N, conn_p, m.B, m.w, x_p)
    assert fp == f and np.array_equal(gp, g[pi])
    # reorder elements: same f and g up to rounding
    perm = np.random.default_rng(2).permutation(m.n_elems)
    fe, ge = orc.mesh_gradient(N, m.conn[perm], m.B[perm], m.w[perm], m.x)
    assert abs(fe - f) <= 1e-13 * abs(f) and rel(ge, g) <= 1e-13
    # x = 0 gives f = 0 and g = 0 exactly
    f0, g0 = orc.mesh_gradient(N, m.conn, m.B, m.w, np.zeros(N))
    assert f0 == 0.0 and not np.any(g0)


def test_degenerate_and_errors(orc):
    # empty element set: f = 0, g = 0
    f, g = orc.mesh_gradient(5, np.zeros((0, 8), np.int32), np.zeros((0, 8)), np.zeros(0),
                             np.ones(5))
    assert f == 0.0 and not np.any(g)
    # a node repeated inside one element contributes twice
    conn = np.array([[0, 0]], np.int32)
    B = np.array([[1.0, 2.0]])
    f, g = orc.mesh_gradient(1, conn, B, np.array([1.0]), np.array([0.5]))
    u = 1.5
    assert abs(g[0] - 3.0 * (u + u / (1 + u * u))) < 1e-15
    # out-of-range connectivity is rejected
    assert orc.mesh_check(4, np.array([[0, 4]], np.int32)) == orc.ERANGE
    assert orc.mesh_check(4, np.array([[-1, 2]], np.int32)) == orc.ERANGE
    with pytest.raises(orc.OracleError):
        orc.mesh_gradient(4, np.array([[0, 9]], np.int32), np.ones((1, 2)), np.ones(1), np.ones(4))


def test_hvp_matches_gradient_differences(orc):
    m = inputs.hex_mesh(8, seed=61)
    d = inputs.fd_directions((m.n_nodes,), 1, seed=62)[0]
    hd = orc.mesh_hvp(m.n_nodes, m.conn, m.B, m.w, m.x, d)
    h = 1e-5
    gp = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x + h * d)[1]
    gm = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x - h * d)[1]
    assert rel(hd, (gp - gm) / (2 * h)) <= 1e-7


# ------------------------------------------------ transposed connectivity

@pytest.mark.parametrize("mesh", [inputs.hex_mesh(10, seed=1), inputs.random_mesh(50, 80, 8, 2),
                                  inputs.chain(33)], ids=["hex10", "rand", "chain"])
def test_csr_bit_exact(orc, mesh):
    offs, inc = orc.mesh_csr(mesh.n_nodes, mesh.conn)
    flat = mesh.conn.ravel().astype(np.int64)
    order = np.argsort(flat, kind="stable")  # ascending node, ties by (e, j)
    want_offs = np.concatenate([[0], np.cumsum(np.bincount(flat, minlength=mesh.n_nodes))])
    assert np.array_equal(offs, want_offs.astype(np.int32))
    assert np.array_equal(inc, order.astype(np.int32))


def test_colour_checker(orc):
    s = 6
    m = inputs.hex_mesh(s, seed=3)
    idx = np.arange(m.n_elems)
    i, j, k = idx % (s - 1), (idx // (s - 1)) % (s - 1), idx // (s - 1) ** 2
    parity = (i % 2 + 2 * (j % 2) + 4 * (k % 2)).astype(np.int32)
    assert orc.colour_conflicts(m.n_nodes, m.conn, parity, 8) == 0
    assert orc.colour_conflicts(m.n_nodes, m.conn, (i % 2).astype(np.int32), 2) > 0


@pytest.mark.parametrize("mesh", [inputs.hex_mesh(20, seed=4), inputs.random_mesh(500, 1200, 5, 3),
                                  inputs.chain(1000)], ids=["hex20", "rand_k5", "chain"])
def test_threaded_oracle_matches_the_plain_one(orc, mesh):
    """The OpenMP build (timed as the CPU baseline) computes the same f and
    gradient; only the summation order differs."""
    f1, g1 = orc.mesh_gradient(mesh.n_nodes, mesh.conn, mesh.B, mesh.w, mesh.x)
    f2, g2, threads = orc.mesh_gradient_threads(mesh.n_nodes, mesh.conn, mesh.B, mesh.w, mesh.x)
    assert threads >= 1
    assert abs(f2 - f1) <= 1e-14 * abs(f1)
    assert rel(g2, g1) <= 1e-14


def _greedy_brute(conn):
    """The greedy colouring's definition taken literally: for every element,
    every earlier element, every pair of corners (pure Python, tiny meshes)."""
    E = conn.shape[0]
    colour = []
    for e in range(E):
        nodes = set(int(v) for v in conn[e])
        taken = {colour[f] for f in range(e) if nodes & set(int(v) for v in conn[f])}
        c = 0
        while c in taken:
            c += 1
        colour.append(c)
    return np.array(colour, dtype=np.int32)


@pytest.mark.parametrize("mesh", [inputs.random_mesh(12, 30, 3, 4), inputs.random_mesh(40, 60, 8, 5),
                                  inputs.random_mesh(6, 15, 5, 6), inputs.hex_mesh(4, seed=2),
                                  inputs.chain(17)],
                         ids=["rand_k3", "rand_k8", "rand_k5_repeats", "hex4", "chain"])
def test_greedy_colour_is_the_definition(orc, mesh):
    colour, nc = orc.greedy_colour(mesh.n_nodes, mesh.conn)
    want = _greedy_brute(mesh.conn)
    assert np.array_equal(colour, want)
    assert nc == int(want.max()) + 1
    assert orc.colour_conflicts(mesh.n_nodes, mesh.conn, colour, nc) == 0


def test_greedy_colour_of_a_structured_hex_is_the_parity_pattern(orc):
    """In lexicographic element order the greedy colouring of a structured hex
    mesh is (i mod 2) + 2 (j mod 2) + 4 (k mod 2): derived by hand for the
    first row pairs and checked here on a 9^3-node mesh."""
    s = 9
    m = inputs.hex_mesh(s, seed=3)
    idx = np.arange(m.n_elems)
    i, j, k = idx % (s - 1), (idx // (s - 1)) % (s - 1), idx // (s - 1) ** 2
    colour, nc = orc.greedy_colour(m.n_nodes, m.conn)
    assert nc == 8
    assert np.array_equal(colour, (i % 2 + 2 * (j % 2) + 4 * (k % 2)).astype(np.int32))
    # a colour bound too small is reported, not truncated
    with pytest.raises(orc.OracleError):
        orc.greedy_colour(m.n_nodes, m.conn, max_colours=7)


# ------------------------------------------------------------------ dense

def test_dot2_exact_rational(orc):
    """Dot2 rows against exact rational arithmetic on ill-conditioned data."""
    rng = np.random.default_rng(7)
    rows, cols = 6, 40
    A = rng.standard_normal((rows, cols)) * np.exp2(rng.integers(-20, 20, (rows, cols)))
    x = rng.standard_normal(cols)
    A[:, -1] = -(A[:, :-1] @ x[:-1]) / x[-1]  # heavy cancellation
    w = np.ones(rows)
    _, r = orc.dense_objective(A, x, w)
    for i in range(rows):
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(A[i], x))
        scale = sum(abs(Fraction(float(a)) * Fraction(float(b))) for a, b in zip(A[i], x))
        # Dot2 bound: |r - exact| <= eps|exact| + gamma_n^2 sum|a b|
        err = abs(Fraction(float(r[i])) - exact)
        assert err <= Fraction(2.3e-16) * abs(exact) + Fraction(1e-28) * scale


def test_dense_vs_blas_and_complex_step(orc):
    d = inputs.dense(300, seed=8, rows=200)
    f, g = orc.dense_gradient(d.A, d.x, d.w)
    r = d.A @ d.x
    assert abs(f - math.fsum(d.w * (0.5 * r * r + 0.5 * np.log1p(r * r)))) <= 1e-12 * abs(f)
    assert rel(g, d.A.T @ (d.w * (r + r / (1 + r * r)))) <= 1e-12
    # complex step on a tiny dense problem
    t = inputs.dense(5, seed=9, rows=4)
    f5, g5 = orc.dense_gradient(t.A, t.x, t.w)
    h = 1e-30
    for i in range(5):
        xc = t.x.astype(complex)
        xc[i] += 1j * h
        rc = t.A @ xc
        fc = sum(t.w[q] * (0.5 * rc[q] ** 2 + 0.5 * cmath.log(1 + rc[q] ** 2)) for q in range(4))
        assert abs(fc.imag / h - g5[i]) <= 1e-14 * max(1.0, abs(g5[i]))
        if i == 0:
            assert abs(fc.real - f5) <= 1e-14 * abs(f5)


def test_dense_fbar_and_shapes(orc):
    d = inputs.dense(64, seed=10, rows=17)
    _, g1 = orc.dense_gradient(d.A, d.x, d.w, 1.0)
    _, g2 = orc.dense_gradient(d.A, d.x, d.w, 2.5)
    assert g1.shape == (64,) and rel(g2, 2.5 * g1) <= 1e-15


# ---------------------------------------------------------- batched dense

def test_bdense_columns_vs_fast_and_dense(orc):
    b = inputs.batched_dense(48, 10, seed=12)
    f, G = orc.bdense_gradient_fast(b.A, b.X, b.W)
    cols = [0, 3, 9]
    fc, Gc = orc.bdense_columns(b.A, b.X, b.W, cols)
    for t, c in enumerate(cols):
        fd, gd = orc.dense_gradient(b.A, b.X[:, c], b.W[:, c])
        assert abs(fc[t] - fd) <= 1e-15 * abs(fd)
        assert rel(Gc[:, t], gd) <= 1e-15
        assert rel(Gc[:, t], G[:, c]) <= 1e-13
    all_f, _ = orc.bdense_columns(b.A, b.X, b.W, list(range(10)))
    assert abs(orc.fsum(all_f) - f) <= 1e-13 * abs(f)


def test_bdense_finite_differences(orc):
    b = inputs.batched_dense(32, 6, seed=13)
    f0, G = orc.bdense_gradient_fast(b.A, b.X, b.W)
    F = lambda X: orc.bdense_gradient_fast(b.A, X, b.W)[0]
    for D in inputs.fd_directions(b.X.shape, 4, seed=33):
        h = 1e-5
        fd = (F(b.X + h * D) - F(b.X - h * D)) / (2 * h)
        assert abs(fd - (G * D).sum()) <= 1e-7 * max(1.0, abs(fd))


# ---------------------------------------------------------- uneven batch

def test_uneven_batch_is_independent_instances(orc):
    bt = inputs.uneven_batch(5, seed=4, lo=3, hi=9)
    assert bt.sides.min() >= 3 and bt.sides.max() <= 9
    fs, g = orc.mesh_batch_gradient(bt)
    for i in range(bt.n_inst):
        m = bt.instance(i)
        f_i, g_i = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
        nn, _, no, _ = bt.inst[i]
        assert fs[i] == f_i and np.array_equal(g[no:no + nn], g_i)
    assert np.array_equal(fs, orc.mesh_batch_objective(bt))


def test_uneven_sides_law():
    s, _ = inputs.uneven_sides(256, seed=4)
    assert s.min() >= 10 and s.max() <= 100
    # log-uniform: the median side is near sqrt(10 * 100)
    assert 22 <= np.median(s) <= 42


# ------------------------------------------- the paper's section 4 example

def _laplacian(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


@pytest.mark.parametrize("n", [1, 2, 3, 17, 1000])
def test_laplace1d_closed_form(orc, n):
    """grad_x f = 6 A (3 A x - b) and grad_b f = -2 (3 A x - b), A symmetric."""
    rng = np.random.default_rng(n)
    x, b = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    f, gx, gb = orc.laplace1d_gradient(x, b)
    A = _laplacian(n)
    y = 3 * (A @ x) - b
    assert abs(f - math.fsum(y * y)) <= 1e-14 * max(f, 1e-300)
    assert rel(gx, 6 * (A @ y)) <= 1e-14
    assert rel(gb, -2 * y) <= 1e-15
    f2, gx2, gb2 = orc.laplace1d_gradient(x, b, fbar=0.5)
    assert rel(gx2, 0.5 * gx) <= 1e-15 and rel(gb2, 0.5 * gb) <= 1e-15


def test_laplace1d_worked_and_complex_step(orc):
    # n = 1: A = [2], y = 6x - b, f = y^2, df/dx = 12 y, df/db = -2 y
    f, gx, gb = orc.laplace1d_gradient([0.25], [0.5])
    assert f == 1.0 and gx[0] == 12.0 and gb[0] == -2.0
    # complex step through an independent evaluation of the example's kernels
    n = 9
    rng = np.random.default_rng(99)
    x, b = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)

    def F(xc, bc):
        xs = [3 * v for v in xc]
        tot = 0j
        for j in range(n):
            y = 2 * xs[j] - bc[j]
            if j != 0:
                y -= xs[j - 1]
            if j != n - 1:
                y -= xs[j + 1]
            tot += y * y
        return tot

    _, gx, gb = orc.laplace1d_gradient(x, b)
    h = 1e-30
    for i in range(n):
        xc = [complex(v) for v in x]
        xc[i] += 1j * h
        assert abs(F(xc, list(b)).imag / h - gx[i]) <= 1e-14 * max(1, abs(gx[i]))
        bc = [complex(v) for v in b]
        bc[i] += 1j * h
        assert abs(F(list(x), bc).imag / h - gb[i]) <= 1e-14 * max(1, abs(gb[i]))
