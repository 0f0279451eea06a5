"""Composed programs on the GPU (pg_prog_*): the generated reverse pass
against the oracle's forward Jacobian accumulation."""
import numpy as np
import pytest
import torch

from oracle import program as OP
from paper_2507_13204_amd import inputs
from paper_2507_13204_amd import pgrad as P

from _helpers import TOL_F64_F, TOL_F64_G, rel, srel, to_dev

pytestmark = pytest.mark.gpu


FUSION = [0, 1]


def run_case(case, grads=True, fusion=1):
    prog = P.Program.from_spec(case.spec, fusion=fusion).plan()
    xs = [to_dev(x) for x in case.inputs]
    out = prog.run(xs, grads=grads)
    torch.cuda.synchronize()
    return prog, out


def check_case(case, fusion=1):
    prog, (f, gs) = run_case(case, fusion=fusion)
    f_ref, g_ref = OP.gradient(case.spec, case.inputs)
    assert srel(f.item(), f_ref) < TOL_F64_F, (case.name, f.item(), f_ref)
    for g, gr in zip(gs, g_ref):
        assert rel(g.cpu().numpy(), gr) < TOL_F64_G, case.name
    return prog


@pytest.mark.parametrize("fusion", FUSION)
@pytest.mark.parametrize("n,E,k,hot", [(1000, 777, 4, 0), (300, 3000, 8, 4), (2500, 513, 3, 0),
                                       (257, 64, 1, 0), (700, 900, 5, 0), (64, 5000, 2, 0)])
def test_mix_program(n, E, k, hot, fusion):
    prog = check_case(inputs.program_mix(n, E, k, seed=7, hot=hot), fusion)
    info = prog.info()
    assert info["atomic_ops"] == 1 and info["rescheduled_ops"] == 1
    assert info["fused_gathers"] == fusion


@pytest.mark.parametrize("fusion", FUSION)
@pytest.mark.parametrize("n", [1, 2, 3, 255, 1000, 10_000])
def test_paper_program(n, fusion, orc):
    case = inputs.program_paper(n, seed=9)
    check_case(case, fusion)
    # and the same numbers as the hand-fused section 4 path
    _, (f, (gx, gb)) = run_case(case, fusion=fusion)
    f2, gx2, gb2 = orc.laplace1d_gradient(*case.inputs)
    assert srel(f.item(), f2) < TOL_F64_F
    assert rel(gx.cpu().numpy(), gx2) < TOL_F64_G and rel(gb.cpu().numpy(), gb2) < TOL_F64_G


@pytest.mark.parametrize("fusion", FUSION)
@pytest.mark.parametrize("s", [2, 9, 17])
def test_mesh_program(s, fusion, orc):
    m = inputs.hex_mesh(s, seed=31)
    case = inputs.program_mesh(m)
    check_case(case, fusion)
    _, (f, (g,)) = run_case(case, fusion=fusion)
    f2, g2 = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    assert srel(f.item(), f2) < TOL_F64_F and rel(g.cpu().numpy(), g2) < TOL_F64_G


@pytest.mark.parametrize("fusion", FUSION)
def test_scan_across_many_chunks(fusion, orc):
    n = 200_003  # 98 scan chunks of 2048 and a ragged tail
    rng = np.random.default_rng(17)
    x = rng.uniform(-1, 1, n)
    w = rng.uniform(0.5, 1.5, n)
    spec = [("input", n), ("scan", 0), ("map", 1, "psi"), ("const", w), ("mul", 2, 3),
            ("sum", 4)]
    case = inputs.ProgramCase(spec, [x], "scan")
    _, (f, (g,)) = run_case(case, fusion=fusion)
    vals = OP.values(spec, [x])
    assert srel(f.item(), vals[-1]) < TOL_F64_F
    idx = [0, 1, 2047, 2048, 4095, 100_000, n - 2, n - 1]
    ref = OP.sampled_gradient(spec, [x], 0, idx)
    got = g.cpu().numpy()
    assert rel(got[idx], ref) < TOL_F64_G
    # every entry: the closed form df/dx_j = sum_{i >= j} w_i psi'(s_i), s the
    # inclusive prefix sum, with the sums in extended precision
    s_ext = np.cumsum(x.astype(np.longdouble))
    v = w * orc.dpsi(s_ext.astype(np.float64))
    closed = np.cumsum(v[::-1].astype(np.longdouble))[::-1].astype(np.float64)
    assert rel(got, closed) < TOL_F64_G


def test_objective_only_and_partial_gradients():
    case = inputs.program_mix(600, 400, 4, seed=8)
    prog = P.Program.from_spec(case.spec).plan()
    xs = [to_dev(x) for x in case.inputs]
    f = prog.run(xs, grads=None)
    f_ref, g_ref = OP.gradient(case.spec, case.inputs)
    assert srel(f.item(), f_ref) < TOL_F64_F
    gy = torch.full_like(xs[1], 7.0)                 # overwritten, not accumulated
    f2, outs = prog.run(xs, grads=[None, gy])
    assert outs[0] is None
    assert rel(gy.cpu().numpy(), g_ref[1]) < TOL_F64_G
    assert srel(f2.item(), f_ref) < TOL_F64_F


def test_repeated_runs_reuse_the_tape():
    case = inputs.program_paper(4097, seed=2)       # no gather: bit-identical reruns
    prog = P.Program.from_spec(case.spec).plan()
    xs = [to_dev(x) for x in case.inputs]
    f1, g1 = prog.run(xs)
    g1 = [g.clone() for g in g1]
    f2, g2 = prog.run(xs)
    torch.cuda.synchronize()
    assert f1.item() == f2.item()
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)


def test_empty_program():
    spec = [("input", 0), ("map", 0, "psi"), ("sum", 1)]
    prog = P.Program.from_spec(spec).plan()
    x = torch.empty(0, dtype=torch.float64, device="cuda")
    f, (g,) = prog.run([x])
    torch.cuda.synchronize()
    assert f.item() == 0.0 and g.numel() == 0


def test_gather_connectivity_is_checked_at_bind():
    conn = np.array([[0, 1], [2, 5]], dtype=np.int32)  # 5 is outside an input of 4
    spec = [("input", 4), ("gather", 0, conn, np.ones((2, 2))), ("sum", 1)]
    with pytest.raises(P.PgError) as e:
        P.Program.from_spec(spec).plan()
    assert e.value.code == P.ERANGE


def _rand(n, seed):
    return np.random.default_rng(seed).uniform(-1, 1, n)


@pytest.mark.parametrize("fusion", FUSION)
def test_sum_of_an_input_and_of_a_gather(fusion):
    n = 1025
    x = _rand(n, 1)
    check_case(inputs.ProgramCase([("input", n), ("sum", 0)], [x], "sum-input"), fusion)
    rng = np.random.default_rng(2)
    conn = rng.integers(0, n, size=(3000, 4)).astype(np.int32)
    B = rng.standard_normal((3000, 4))
    check_case(inputs.ProgramCase([("input", n), ("gather", 0, conn, B), ("sum", 1)], [x],
                                  "sum-gather"), fusion)


@pytest.mark.parametrize("fusion", FUSION)
def test_gather_whose_operand_the_group_also_reads(fusion):
    # E == n: the group reads x both through the gather and directly, so the
    # gather must not be fused (a store and atomics into one shadow).
    n = 2000
    rng = np.random.default_rng(3)
    x = _rand(n, 4)
    conn = rng.integers(0, n, size=(n, 8)).astype(np.int32)
    B = rng.standard_normal((n, 8)) / 3
    spec = [("input", n), ("gather", 0, conn, B), ("mul", 1, 0), ("map", 2, "psi"), ("sum", 3)]
    prog = check_case(inputs.ProgramCase(spec, [x], "gather-and-leaf"), fusion)
    assert prog.info()["fused_gathers"] == 0


@pytest.mark.parametrize("fusion", FUSION)
def test_long_chain_and_many_leaves(fusion):
    # 20 pointwise constructs over 10 inputs: more than one group's slots,
    # leaves and ops, so the planner has to split.
    n = 3001
    xs = [_rand(n, 10 + i) for i in range(10)]
    spec = [("input", n) for _ in range(10)]
    cur = 0
    for i in range(1, 10):
        spec.append(("add", cur, 0.9, i, 0.3))
        cur = len(spec) - 1
        spec.append(("map", cur, "psi" if i % 2 else "square"))
        cur = len(spec) - 1
        spec.append(("scale", cur, 0.5))
        cur = len(spec) - 1
    spec.append(("mul", cur, cur))
    spec.append(("sum", len(spec) - 1))
    prog = check_case(inputs.ProgramCase(spec, xs, "long-chain"), fusion)
    if fusion:
        assert prog.info()["groups"] > 1


@pytest.mark.parametrize("fusion", FUSION)
def test_self_add_and_shared_leaf(fusion):
    n = 777
    x, y = _rand(n, 5), _rand(n, 6)
    spec = [("input", n), ("input", n), ("add", 0, 1.5, 0, -0.25), ("mul", 2, 1),
            ("stencil", 3, [0, -1], [1.0, 0.5]), ("add", 4, 1.0, 3, 1.0), ("mul", 5, 0),
            ("sum", 6)]
    check_case(inputs.ProgramCase(spec, [x, y], "self-add"), fusion)


@pytest.mark.parametrize("fusion", FUSION)
@pytest.mark.parametrize("n_seg,mean", [(1000, 20.0), (37, 300.0), (5, 0.5)])
def test_segment_sum_and_broadcast(n_seg, mean, fusion):
    check_case(inputs.program_segments(n_seg, mean, seed=21), fusion)


def test_segment_offsets_are_checked_at_bind():
    off = np.array([0, 3, 2, 5], dtype=np.int64)          # decreasing
    spec = [("input", 5), ("segsum", 0, off), ("sum", 1)]
    with pytest.raises(P.PgError) as e:
        P.Program.from_spec(spec).plan()
    assert e.value.code == P.ERANGE
    off = np.array([0, 2, 4], dtype=np.int64)             # ends short of the input
    spec = [("input", 5), ("segsum", 0, off), ("sum", 1)]
    with pytest.raises(P.PgError) as e:
        P.Program.from_spec(spec).plan()
    assert e.value.code == P.ERANGE


@pytest.mark.parametrize("fusion", FUSION)
def test_broadcast_with_no_outputs(fusion):
    # every segment empty: the broadcast has no outputs, yet its reverse must
    # still define the adjoint of each segment (zero)
    off = np.zeros(4, dtype=np.int64)
    x = _rand(3, 9)
    spec = [("input", 3), ("bcast", 0, off), ("sum", 1)]
    prog, (f, (g,)) = run_case(inputs.ProgramCase(spec, [x], "empty-bcast"), fusion=fusion)
    assert f.item() == 0.0
    assert torch.equal(g.cpu(), torch.zeros(3, dtype=torch.float64))


@pytest.mark.parametrize("fusion", FUSION)
def test_mesh_program_full_size(fusion, orc):
    """The 128^3 element objective as constructs, in the benchmark's launch
    configuration, against the mesh oracle (pinned to the program oracle at
    small sizes)."""
    m = inputs.hex_mesh(128)
    case = inputs.program_mesh(m)
    prog, (f, (g,)) = run_case(case, fusion=fusion)
    f_ref, g_ref = orc.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    assert srel(f.item(), f_ref) < TOL_F64_F
    assert rel(g.cpu().numpy(), g_ref) < TOL_F64_G
    if fusion:
        assert prog.info()["fwd_kernels"] == 2 and prog.info()["rev_kernels"] == 0


@pytest.mark.parametrize("fusion", FUSION)
def test_seeded_run_scales_the_gradient(fusion):
    case = inputs.program_mix(700, 500, 4, seed=13)
    prog = P.Program.from_spec(case.spec, fusion=fusion).plan()
    xs = [to_dev(x) for x in case.inputs]
    f1, g1 = prog.run(xs)
    fbar = torch.tensor([-2.5], dtype=torch.float64, device="cuda")
    f2, g2 = prog.run(xs, fbar=fbar)
    torch.cuda.synchronize()
    assert f1.item() == f2.item()          # the seed scales gradients only
    for a, b in zip(g1, g2):
        assert rel(b.cpu().numpy(), -2.5 * a.cpu().numpy()) < 1e-15


def test_program_autograd_matches_oracle_and_fd():
    case = inputs.program_paper(300, seed=4)
    prog = P.Program.from_spec(case.spec).plan()
    x, b = [to_dev(v).requires_grad_(True) for v in case.inputs]
    f = P.ProgramFn.apply(prog, x, b)
    (3.0 * f).backward()
    _, (gx_ref, gb_ref) = OP.gradient(case.spec, case.inputs)
    assert rel(x.grad.cpu().numpy(), 3.0 * gx_ref) < TOL_F64_G
    assert rel(b.grad.cpu().numpy(), 3.0 * gb_ref) < TOL_F64_G
    # central differences of the objective along random directions
    rng = np.random.default_rng(8)
    for _ in range(4):
        d = rng.standard_normal(300)
        h = 1e-5
        xp, xm = case.inputs[0] + h * d, case.inputs[0] - h * d
        fp = prog.run([to_dev(xp), to_dev(case.inputs[1])], grads=None).item()
        fm = prog.run([to_dev(xm), to_dev(case.inputs[1])], grads=None).item()
        fd = (fp - fm) / (2 * h)
        assert abs(fd - float(gx_ref @ d)) <= 1e-6 * max(1.0, abs(fd))


def test_program_run_replays_from_a_graph():
    """A fused program run (objective and gradient) captured in a HIP graph
    and replayed; every replay matches the eager result."""
    case = inputs.program_mix(1000, 777, 4, seed=7)
    prog = P.Program.from_spec(case.spec).plan()
    xs = [to_dev(x) for x in case.inputs]
    f_e, g_e = prog.run(xs)
    torch.cuda.synchronize()
    f = torch.empty((), dtype=torch.float64, device="cuda")
    gs = [torch.empty_like(x) for x in xs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        prog.run(xs, grads=gs, f_out=f, stream=s)
        with torch.cuda.graph(graph, stream=s):
            prog.run(xs, grads=gs, f_out=f, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        f.fill_(float("nan"))
        for g in gs:
            g.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert srel(f.item(), f_e.item()) < 1e-14
        for a, b in zip(gs, g_e):
            assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-13


@pytest.mark.parametrize("n", [300, 16_384, 16_385])
def test_small_sum_reduced_by_its_last_workgroup(n):
    """Up to 64 summing workgroups (16,384 summed entries) the sum group's last
    workgroup reduces f through a ticket it re-arms; objective-only and
    gradient runs alternate on one plan and every f is the same, bitwise, and
    the oracle's; one more entry takes the separate reduction launch."""
    case = inputs.program_paper(n, seed=21)
    prog = P.Program.from_spec(case.spec).plan()
    xs = [to_dev(x) for x in case.inputs]
    f_ref, g_ref = OP.gradient(case.spec, case.inputs)
    fs = []
    for i in range(4):
        if i % 2 == 0:
            f, gs = prog.run(xs, grads=True)
            for g, gr in zip(gs, g_ref):
                assert rel(g.cpu().numpy(), gr) < TOL_F64_G
        else:
            f = prog.run(xs, grads=False)
        fs.append(f.item())
    assert srel(fs[0], f_ref) < TOL_F64_F
    assert all(v == fs[0] for v in fs)
    # the fused reduction saves the launch (forward: the stencil and the group)
    assert prog.info()["fwd_kernels"] == (2 if n <= 16_384 else 3)
