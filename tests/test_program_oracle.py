"""Pins of the composed-program oracle (forward Jacobian accumulation) against
facts that do not come from it: the complex-step derivative of its own
forward values, closed forms, and the independently pinned mesh and
section 4 oracles."""
import numpy as np
import pytest

from oracle import program as OP
from paper_2507_13204_amd import inputs

from _helpers import rel, srel


def test_complex_step_pins_every_gradient_entry():
    # Every construct appears; a transposed stencil or gather Jacobian, a
    # dropped product-rule term or a wrong scan direction changes some entry.
    case = inputs.program_mix(23, 17, 3, seed=11)
    f, grads = OP.gradient(case.spec, case.inputs)
    assert np.isfinite(f)
    for which, x in enumerate(case.inputs):
        cs = np.array([OP.complex_step(case.spec, case.inputs, which, j) for j in range(x.size)])
        assert rel(grads[which], cs) < 1e-13, which


def test_complex_step_hot_gather():
    case = inputs.program_mix(19, 40, 4, seed=12, hot=3)
    _, grads = OP.gradient(case.spec, case.inputs)
    cs = np.array([OP.complex_step(case.spec, case.inputs, 0, j) for j in range(19)])
    assert rel(grads[0], cs) < 1e-13


def test_mesh_program_matches_mesh_oracle(orc):
    m = inputs.random_mesh(60, 45, 4, seed=21)
    case = inputs.program_mesh(m)
    f, (g,) = OP.gradient(case.spec, case.inputs)
    f_ref, g_ref = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    assert srel(f, f_ref) < 1e-14
    assert rel(g, g_ref) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 37])
def test_paper_program_matches_closed_form_and_oracle(orc, n):
    case = inputs.program_paper(n, seed=3)
    x, b = case.inputs
    f, (gx, gb) = OP.gradient(case.spec, case.inputs)
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    r = 3.0 * (A @ x) - b
    assert srel(f, float(r @ r)) < 1e-13
    assert rel(gx, 6.0 * (A @ r)) < 1e-13
    assert rel(gb, -2.0 * r) < 1e-13
    f2, gx2, gb2 = orc.laplace1d_gradient(x, b)
    assert srel(f, f2) < 1e-13 and rel(gx, gx2) < 1e-13 and rel(gb, gb2) < 1e-13


def test_scan_gradient_is_reverse_cumulative_sum():
    rng = np.random.default_rng(4)
    n = 31
    x = rng.uniform(-1, 1, n)
    w = rng.uniform(0.5, 1.5, n)
    spec = [("input", n), ("scan", 0), ("const", w), ("mul", 1, 2), ("sum", 3)]
    f, (g,) = OP.gradient(spec, [x])
    # d/dx_j sum_i w_i sum_{l <= i} x_l = sum_{i >= j} w_i
    assert rel(g, np.cumsum(w[::-1])[::-1]) < 1e-15
    assert srel(f, float(w @ np.cumsum(x))) < 1e-14


def test_self_product_and_stencil_quadratic():
    rng = np.random.default_rng(5)
    n = 12
    x = rng.uniform(-1, 1, n)
    offs, coef = [-1, 2], [0.5, -1.5]
    spec = [("input", n), ("stencil", 0, offs, coef), ("mul", 1, 1), ("sum", 2)]
    S = np.zeros((n, n))
    for o, c in zip(offs, coef):
        for i in range(n):
            if 0 <= i + o < n:
                S[i, i + o] += c
    f, (g,) = OP.gradient(spec, [x])
    assert srel(f, float((S @ x) @ (S @ x))) < 1e-14
    assert rel(g, 2.0 * S.T @ (S @ x)) < 1e-14


def test_inactive_branch_contributes_nothing():
    rng = np.random.default_rng(6)
    n = 9
    x, c = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    spec = [("input", n), ("const", c), ("map", 1, "psi"), ("add", 0, 2.0, 2, 1.0), ("sum", 3)]
    f, (g,) = OP.gradient(spec, [x])
    assert np.array_equal(g, np.full(n, 2.0))


def test_psi_map_matches_oracle_psi(orc):
    s = np.linspace(-3, 3, 101)
    spec = [("input", 101), ("map", 0, "psi"), ("sum", 1)]
    vals = OP.values(spec, [s])
    assert rel(vals[1], orc.psi(s)) < 1e-15
    _, (g,) = OP.gradient(spec, [s])
    assert rel(g, orc.dpsi(s)) < 1e-15


def test_segments_complex_step():
    case = inputs.program_segments(9, 3.0, seed=13)
    assert (np.diff(case.spec[1][2]) == 0).any()      # an empty segment is present
    _, (g,) = OP.gradient(case.spec, case.inputs)
    cs = np.array([OP.complex_step(case.spec, case.inputs, 0, j) for j in range(case.inputs[0].size)])
    assert rel(g, cs) < 1e-13


def test_broadcast_of_segment_sum_closed_form():
    off = inputs.segment_offsets(12, 4.0, seed=14)
    n = int(off[-1])
    rng = np.random.default_rng(15)
    x, w = rng.uniform(-1, 1, n), rng.uniform(0.5, 1.5, n)
    spec = [("input", n), ("segsum", 0, off), ("bcast", 1, off), ("const", w), ("mul", 2, 3),
            ("sum", 4)]
    f, (g,) = OP.gradient(spec, [x])
    seg = np.repeat(np.arange(12), np.diff(off))
    sx = np.bincount(seg, weights=x, minlength=12)
    sw = np.bincount(seg, weights=w, minlength=12)
    # f = sum_i w_i * (sum of x over i's segment); df/dx_i = sum of w over i's segment
    assert srel(f, float(w @ sx[seg])) < 1e-14
    assert rel(g, sw[seg]) < 1e-14
