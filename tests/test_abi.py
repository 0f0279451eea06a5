"""The C-ABI library loads, exports what include/pgrad.h declares, and
rejects bad arguments before touching the GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2507_13204_amd import pgrad as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pgrad.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(pg_[a-z_0-9]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_bound_entry_points():
    decl = declared_functions()
    assert set(decl) == set(P.EXPORTS), (decl, P.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = P.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.pg_version() == 2


def test_default_options():
    o = P.lib().pg_default_options()
    assert (o.adjoint, o.ckpt, o.block, o.tile, o.accumulate, o.scatter) == (0, 0, 0, 0, 0, 0)
    assert (o.onepass, o.reserved, o.tape_budget) == (0, 0, 0)
    assert ctypes.sizeof(P.Options) == 40  # 8 int32 (one reserved) + one int64


def _info(plan):
    st = P.PlanInfo()
    assert P.lib().pg_plan_info(plan, ctypes.byref(st)) == P.OK
    return st


@pytest.mark.parametrize("budget,expect", [(900 * 8, P.STORE), (900 * 8 - 1, P.RECOMPUTE),
                                           (1 << 40, P.STORE)])
def test_ckpt_auto_is_chosen_by_the_tape_budget(budget, expect):
    """PG_CKPT_AUTO stores the tape (u_e, 8 bytes per element) when it fits the
    caller's budget and recomputes otherwise; the choice is visible in
    pg_plan_info and in the workspace size (the stored tape lives there)."""
    opts = P.make_options(ckpt="auto", onepass=False, tape_budget=budget)
    st, plan, ws = plan_mesh(n_nodes=1000, n_elems=900, k=8, opts=opts)
    assert st == P.OK
    info = _info(plan)
    assert info.ckpt == expect and info.tape_bytes == 900 * 8 and info.tape_budget == budget
    assert info.bound == 0 and info.lds_slots == 0 and info.kind == 1
    _, ref, ws_ref = plan_mesh(n_nodes=1000, n_elems=900, k=8,
                               opts=P.make_options(ckpt=["recompute", "store"][expect],
                                                   onepass=False))
    assert ws == ws_ref
    sz = ctypes.c_size_t()
    assert P.lib().pg_tape_bytes(plan, ctypes.byref(sz)) == P.OK and sz.value == 900 * 8
    P.lib().pg_plan_destroy(plan)
    P.lib().pg_plan_destroy(ref)


def test_bdense_tape_is_v_and_dense_has_none():
    L = P.lib()
    plan = ctypes.c_void_p()
    sz = ctypes.c_size_t()
    o = P.make_options(ckpt="auto", tape_budget=64 * 32 * 4)
    assert L.pg_bdense_plan(ctypes.byref(plan), 64, 32, FAKE, FAKE, P.F32, ctypes.byref(o),
                            ctypes.byref(sz)) == P.OK
    assert _info(plan).ckpt == P.STORE
    t = ctypes.c_size_t()
    assert L.pg_tape_bytes(plan, ctypes.byref(t)) == P.OK and t.value == 64 * 32 * 4
    L.pg_plan_destroy(plan)
    assert L.pg_dense_plan(ctypes.byref(plan), 100, 50, FAKE, FAKE, P.F64, ctypes.byref(o),
                           ctypes.byref(sz)) == P.OK
    assert _info(plan).ckpt == P.RECOMPUTE  # nothing to store
    assert L.pg_tape_bytes(plan, ctypes.byref(t)) == P.EUNSUPPORTED
    L.pg_plan_destroy(plan)


@pytest.mark.parametrize("field,value", [("reserved", 1), ("tape_budget", -1), ("ckpt", 3)])
def test_bad_checkpoint_options(field, value):
    o = P.make_options()
    setattr(o, field, value)
    st, plan, _ = plan_mesh(opts=o)
    assert st == P.EINVAL and not plan.value


def test_tape_calls_and_exports_need_a_bound_plan():
    st, plan, _ = plan_mesh(opts=P.make_options(ckpt="store"))
    L = P.lib()
    assert L.pg_objective_tape(plan, FAKE, FAKE, FAKE, None) == P.ESTATE
    assert L.pg_adjoint_tape(plan, FAKE, FAKE, FAKE, None) == P.ESTATE
    sz = ctypes.c_size_t()
    assert L.pg_plan_export(plan, P.EXPORT_CSR_OFFS, None, 0, ctypes.byref(sz)) == P.ESTATE
    L.pg_plan_destroy(plan)


def test_scale_argument_checks():
    L = P.lib()
    assert L.pg_scale(7, 10, FAKE, FAKE, FAKE, None) == P.EDTYPE
    assert L.pg_scale(P.F64, -1, FAKE, FAKE, FAKE, None) == P.EINVAL
    assert L.pg_scale(P.F64, 10, None, FAKE, FAKE + 4096, None) == P.EINVAL
    assert L.pg_scale(P.F64, 10, FAKE + 8192, FAKE, None, None) == P.EINVAL
    # y overlapping x without being x
    assert L.pg_scale(P.F64, 10, FAKE + 8192, FAKE, FAKE + 8, None) == P.EALIAS
    assert L.pg_scale(P.F32, 10, FAKE + 4096 + 16, FAKE, FAKE + 4096, None) == P.EALIAS
    # n = 0 enqueues nothing
    assert L.pg_scale(P.F64, 0, FAKE, None, None, None) == P.OK


FAKE = 1 << 20  # an aligned non-null address; plan creation never dereferences it


def plan_mesh(n_nodes=10, n_elems=4, k=8, conn=FAKE, B=FAKE, w=FAKE, dtype=P.F64, opts=None):
    L = P.lib()
    plan = ctypes.c_void_p()
    sz = ctypes.c_size_t()
    o = opts if opts is not None else P.make_options()
    st = L.pg_mesh_plan(ctypes.byref(plan), n_nodes, n_elems, k, conn, B, w, dtype,
                        ctypes.byref(o), ctypes.byref(sz))
    return st, plan, sz.value


def test_mesh_plan_is_host_only_and_sizes_workspace():
    st, plan, ws = plan_mesh(n_nodes=1000, n_elems=900, k=8, opts=P.make_options(onepass=False))
    assert st == P.OK and ws > 0 and ws % P.WORKSPACE_ALIGN == 0
    st2, plan2, ws2 = plan_mesh(n_nodes=1000, n_elems=900, k=8,
                                opts=P.make_options("gather", "store"))
    assert st2 == P.OK
    # the transposed connectivity and the tape make the workspace larger
    assert ws2 >= ws + 900 * 8 * 4 + 900 * 8 * 2
    L = P.lib()
    # unbound plans refuse to evaluate
    assert L.pg_objective(plan, FAKE, FAKE, None) == P.ESTATE
    assert b"pg_bind_workspace" in L.pg_last_error()
    # workspace checks happen before any HIP call
    assert L.pg_bind_workspace(plan, None, ws, None) == P.EWORKSPACE
    assert L.pg_bind_workspace(plan, FAKE, ws - 1, None) == P.EWORKSPACE
    assert L.pg_bind_workspace(plan, FAKE + 8, ws, None) == P.EWORKSPACE
    assert L.pg_plan_destroy(plan) == P.OK
    assert L.pg_plan_destroy(plan2) == P.OK


@pytest.mark.parametrize("kw,code", [
    (dict(n_nodes=-1), P.EINVAL),
    (dict(n_elems=-3), P.EINVAL),
    (dict(k=0), P.EINVAL),
    (dict(k=33), P.EINVAL),
    (dict(n_nodes=1 << 31), P.EINVAL),
    (dict(n_elems=(1 << 28), k=8), P.EINVAL),
    (dict(conn=None), P.EINVAL),
    (dict(B=FAKE + 4), P.EINVAL),
    (dict(dtype=7), P.EDTYPE),
    (dict(n_nodes=0, n_elems=3), P.ERANGE),
    (dict(opts="bad_adjoint"), P.EINVAL),
    (dict(opts="bad_block"), P.EINVAL),
    (dict(opts="bad_tile"), P.EINVAL),
    (dict(opts="bad_scatter"), P.EINVAL),
    (dict(opts="bad_onepass"), P.EINVAL),
])
def test_mesh_plan_argument_errors(kw, code):
    if kw.get("opts") == "bad_adjoint":
        kw["opts"] = P.make_options(adjoint=9)
    elif kw.get("opts") == "bad_block":
        kw["opts"] = P.make_options(block=100)
    elif kw.get("opts") == "bad_tile":
        kw["opts"] = P.make_options(tile=3)
    elif kw.get("opts") == "bad_scatter":
        kw["opts"] = P.make_options(scatter=4)
    elif kw.get("opts") == "bad_onepass":
        kw["opts"] = P.make_options()
        kw["opts"].onepass = 2
    st, plan, _ = plan_mesh(**kw)
    assert st == code
    assert not plan.value
    assert len(P.lib().pg_last_error()) > 0


@pytest.mark.parametrize("n_nodes,n_elems,k,adjoint,small", [
    (2000, 1000, 8, "atomic", True),        # 2 workgroups of 512, 2,000 nodes
    (10_000, 9_999, 2, "atomic", True),     # the 1D chain of 10^4 nodes
    (16_384, 32_768, 4, "atomic", True),    # 64 workgroups and 16,384 nodes: the limits
    (16_385, 1000, 8, "atomic", False),     # one node too many
    (2000, 32_769, 8, "atomic", False),     # 65 workgroups
    (2000, 1000, 5, "atomic", False),       # k not held in registers
    (2000, 1000, 8, "gather", False),       # not the atomic adjoint
])
def test_one_launch_plans_take_a_node_buffer(n_nodes, n_elems, k, adjoint, small):
    """A small mesh's plan (atomic adjoint, k = 2, 4 or 8, at most 64
    workgroups and 16,384 nodes) holds an FP64 buffer of n_nodes entries and a
    ticket for its one-launch calls; onepass = 1 or any larger mesh does not."""
    st, plan, ws = plan_mesh(n_nodes=n_nodes, n_elems=n_elems, k=k,
                             opts=P.make_options(adjoint=adjoint))
    st2, plan2, ws_off = plan_mesh(n_nodes=n_nodes, n_elems=n_elems, k=k,
                                   opts=P.make_options(adjoint=adjoint, onepass=False))
    assert st == P.OK and st2 == P.OK
    if small:
        assert ws - ws_off >= 8 * n_nodes
    else:
        assert ws == ws_off
    P.lib().pg_plan_destroy(plan)
    P.lib().pg_plan_destroy(plan2)


def test_empty_mesh_plan_is_valid():
    st, plan, ws = plan_mesh(n_nodes=5, n_elems=0, conn=None, B=None, w=None)
    assert st == P.OK
    P.lib().pg_plan_destroy(plan)


def test_dense_and_bdense_plans():
    L = P.lib()
    plan = ctypes.c_void_p()
    sz = ctypes.c_size_t()
    o = P.make_options()
    assert L.pg_dense_plan(ctypes.byref(plan), 100, 50, FAKE, FAKE, P.F64, ctypes.byref(o),
                           ctypes.byref(sz)) == P.OK
    L.pg_plan_destroy(plan)
    assert L.pg_dense_plan(ctypes.byref(plan), -1, 50, FAKE, FAKE, P.F64, ctypes.byref(o),
                           ctypes.byref(sz)) == P.EINVAL
    assert L.pg_bdense_plan(ctypes.byref(plan), 64, 32, FAKE, FAKE, P.F32, ctypes.byref(o),
                            ctypes.byref(sz)) == P.OK
    # the stored tape V is m x n in the plan dtype
    assert sz.value >= 64 * 32 * 4
    L.pg_plan_destroy(plan)
    assert L.pg_bdense_plan(ctypes.byref(plan), 64, 32, FAKE + 4, FAKE, P.F32, ctypes.byref(o),
                            ctypes.byref(sz)) == P.EINVAL


def test_batch_plan_validation():
    L = P.lib()
    plan = ctypes.c_void_p()
    sz = ctypes.c_size_t()
    o = P.make_options("atomic")
    arr = (P.Instance * 2)(P.Instance(27, 8, 0, 0), P.Instance(64, 27, 27, 8))
    assert L.pg_mesh_batch_plan(ctypes.byref(plan), 2, arr, 8, FAKE, FAKE, FAKE, P.F64,
                                ctypes.byref(o), ctypes.byref(sz)) == P.OK
    L.pg_plan_destroy(plan)
    bad = (P.Instance * 1)(P.Instance(-1, 8, 0, 0))
    assert L.pg_mesh_batch_plan(ctypes.byref(plan), 1, bad, 8, FAKE, FAKE, FAKE, P.F64,
                                ctypes.byref(o), ctypes.byref(sz)) == P.EINVAL
    og = P.make_options("gather")
    assert L.pg_mesh_batch_plan(ctypes.byref(plan), 2, arr, 8, FAKE, FAKE, FAKE, P.F64,
                                ctypes.byref(og), ctypes.byref(sz)) == P.EUNSUPPORTED


def test_timing_arguments():
    st, plan, _ = plan_mesh()
    L = P.lib()
    assert L.pg_timing(plan, 5) == P.EINVAL
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    assert L.pg_timing(plan, 0) == P.OK
    assert L.pg_timing_read(plan, ctypes.byref(ms), ctypes.byref(n)) == P.OK and n.value == 0
    L.pg_plan_destroy(plan)


# ---------------------------------------------------------- composed programs

def _prog():
    L = P.lib()
    p = ctypes.c_void_p()
    assert L.pg_prog_create(ctypes.byref(p)) == P.OK
    return L, p


def _v(fn, *args):
    v = ctypes.c_int32(-1)
    st = fn(*args, ctypes.byref(v))
    return st, v.value


def test_program_builders_check_their_arguments():
    L, p = _prog()
    st, x = _v(L.pg_prog_input, p, 100)
    assert st == P.OK and x == 0
    st, y = _v(L.pg_prog_input, p, 50)
    assert st == P.OK and y == 1
    assert _v(L.pg_prog_scale, p, 7, 1.0)[0] == P.EINVAL            # no such view
    assert _v(L.pg_prog_add, p, x, 1.0, y, 1.0)[0] == P.EINVAL      # lengths differ
    assert _v(L.pg_prog_mul, p, x, y)[0] == P.EINVAL
    off = (ctypes.c_int32 * 17)(*range(17))
    cf = (ctypes.c_double * 17)(*([1.0] * 17))
    assert _v(L.pg_prog_stencil, p, x, 17, off, cf)[0] == P.EINVAL  # too many taps
    assert _v(L.pg_prog_stencil, p, x, 0, off, cf)[0] == P.EINVAL
    assert _v(L.pg_prog_map, p, x, 9)[0] == P.EINVAL                # unknown map
    assert _v(L.pg_prog_gather, p, x, 10, 0, FAKE, FAKE)[0] == P.EINVAL   # k < 1
    assert _v(L.pg_prog_gather, p, x, 10, 33, FAKE, FAKE)[0] == P.EINVAL  # k > 32
    assert _v(L.pg_prog_gather, p, x, 10, 4, None, FAKE)[0] == P.EINVAL
    assert _v(L.pg_prog_const, p, 5, None)[0] == P.EINVAL
    assert L.pg_prog_plan(p, ctypes.byref(ctypes.c_size_t())) == P.ESTATE  # no sum yet
    assert L.pg_prog_sum(p, x) == P.OK
    assert L.pg_prog_sum(p, x) == P.ESTATE
    assert _v(L.pg_prog_scale, p, x, 2.0)[0] == P.ESTATE            # program ended
    L.pg_prog_destroy(p)


def test_program_plan_reports_the_generated_reverse_pass():
    """Host-only planning: activity analysis, race rule and tape size."""
    L, p = _prog()
    n, E, k = 1000, 300, 4
    _, x = _v(L.pg_prog_input, p, n)
    _, c = _v(L.pg_prog_const, p, n, FAKE)
    off = (ctypes.c_int32 * 3)(-1, 0, 1)
    cf = (ctypes.c_double * 3)(-1.0, 2.0, -1.0)
    _, s1 = _v(L.pg_prog_stencil, p, x, 3, off, cf)       # active, 3 taps: rescheduled
    _, s2 = _v(L.pg_prog_stencil, p, c, 3, off, cf)       # inactive: no reverse kernel
    _, a = _v(L.pg_prog_add, p, s1, 1.0, s2, -1.0)
    _, g = _v(L.pg_prog_gather, p, a, E, k, FAKE, FAKE)   # active gather: atomic
    _, gc = _v(L.pg_prog_gather, p, c, E, k, FAKE, FAKE)  # inactive gather
    _, m = _v(L.pg_prog_mul, p, g, gc)
    _, sc = _v(L.pg_prog_scan, p, m)
    _, q = _v(L.pg_prog_map, p, sc, 0)
    assert L.pg_prog_sum(p, q) == P.OK
    sz = ctypes.c_size_t()
    assert L.pg_prog_plan(p, ctypes.byref(sz)) == P.OK
    assert sz.value > 0 and sz.value % P.WORKSPACE_ALIGN == 0
    st = P.ProgStats()
    assert L.pg_prog_info(p, ctypes.byref(st)) == P.OK
    # Groups: {a} (sealed when the gather g reads it), {m} (sealed by the scan),
    # {q + sum}.  The gather g is read only by group {m} and runs inside it;
    # gc, read by the same group, runs in a group of its own.
    assert st.groups == 4 and st.fused_gathers == 1 and st.dead_ops == 0
    # forward: s1, s2, gc, the scan's 3, three groups; the final reduction is
    # the sum group's last workgroup (300 summed entries: at most 64 workgroups)
    assert st.fwd_kernels == 3 + 3 + 3
    # reverse: s1, the scan's 3, groups {a} and {m}; inactive s2 and gc have
    # none; the sum group runs its reverse inside its forward launch
    assert st.rev_kernels == 1 + 3 + 2
    assert st.atomic_ops == 1 and st.rescheduled_ops == 1
    # recorded: s1, s2, gc, the scan (stand-alone outputs), a and m (exports)
    assert st.tape_bytes == 8 * (3 * n + 3 * E)
    assert sz.value == st.workspace_bytes
    # plus shadows of s1, a, m, the scan and the input
    assert sz.value >= st.tape_bytes + 8 * (3 * n + 2 * E)
    # binding checks size and alignment before any device work
    assert L.pg_prog_bind_workspace(p, None, sz.value) == P.EWORKSPACE
    assert L.pg_prog_bind_workspace(p, FAKE + 8, sz.value) == P.EWORKSPACE
    assert L.pg_prog_bind_workspace(p, FAKE, sz.value - 1) == P.EWORKSPACE
    ins = (ctypes.c_void_p * 1)(FAKE)
    assert L.pg_prog_run(p, ins, None, None, None, None) == P.ESTATE  # no workspace bound
    L.pg_prog_destroy(p)


def _mesh_program(L, p, n=500, E=400, k=8):
    _, x = _v(L.pg_prog_input, p, n)
    _, u = _v(L.pg_prog_gather, p, x, E, k, FAKE, FAKE)
    _, s = _v(L.pg_prog_map, p, u, 1)
    _, w = _v(L.pg_prog_const, p, E, FAKE)
    _, t = _v(L.pg_prog_mul, p, s, w)
    _, dead = _v(L.pg_prog_scale, p, t, 2.0)          # feeds nothing
    assert L.pg_prog_sum(p, t) == P.OK


@pytest.mark.parametrize("fusion", [0, 1])
def test_mesh_program_plan(fusion):
    L, p = _prog()
    assert L.pg_prog_fusion(p, fusion) == P.OK
    _mesh_program(L, p)
    sz = ctypes.c_size_t()
    assert L.pg_prog_plan(p, ctypes.byref(sz)) == P.OK
    st = P.ProgStats()
    assert L.pg_prog_info(p, ctypes.byref(st)) == P.OK
    assert st.dead_ops == 1 and st.atomic_ops == 1
    if fusion:
        # gather -> map -> mul -> sum is one kernel computing f and the gradient
        # (its last workgroup sums the partials)
        assert (st.groups, st.fused_gathers, st.fwd_kernels, st.rev_kernels) == (1, 1, 1, 0)
        assert st.tape_bytes == 0
    else:
        # one kernel per construct (the gather in a group of its own, the sum's
        # partials taken by the mul kernel), then the final reduction; reverse:
        # mul (seeded), map, the gather's atomic scatter; recorded: the
        # gather's and the map's outputs
        assert (st.groups, st.fused_gathers, st.fwd_kernels, st.rev_kernels) == (3, 0, 4, 3)
        assert st.tape_bytes == 8 * 2 * 400
    L.pg_prog_destroy(p)


@pytest.mark.parametrize("fusion", [0, 1])
def test_scale_folds_into_the_stencil_that_reads_it(fusion):
    """The section 4 example as constructs: with fusion the scale by 3 folds
    into the stencil's coefficients, so the forward pass is the stencil and
    the group (subtract b, square, sum; its last workgroup also reduces f),
    and the reverse the rescheduled stencil; a scale with a second reader
    does not fold."""
    L, p = _prog()
    assert L.pg_prog_fusion(p, fusion) == P.OK
    n = 1000
    _, x = _v(L.pg_prog_input, p, n)
    _, b = _v(L.pg_prog_input, p, n)
    _, sx = _v(L.pg_prog_scale, p, x, 3.0)
    off = (ctypes.c_int32 * 3)(-1, 0, 1)
    cf = (ctypes.c_double * 3)(-1.0, 2.0, -1.0)
    _, y = _v(L.pg_prog_stencil, p, sx, 3, off, cf)
    _, r = _v(L.pg_prog_add, p, y, 1.0, b, -1.0)
    _, q = _v(L.pg_prog_map, p, r, 0)
    assert L.pg_prog_sum(p, q) == P.OK
    sz = ctypes.c_size_t()
    assert L.pg_prog_plan(p, ctypes.byref(sz)) == P.OK
    st = P.ProgStats()
    assert L.pg_prog_info(p, ctypes.byref(st)) == P.OK
    assert st.dead_ops == 0 and st.rescheduled_ops == 1
    if fusion:
        assert (st.folded_ops, st.groups, st.fwd_kernels, st.rev_kernels) == (1, 1, 2, 1)
    else:
        assert (st.folded_ops, st.groups, st.fwd_kernels, st.rev_kernels) == (0, 3, 5, 4)
    L.pg_prog_destroy(p)
    # a second reader of the scale keeps it
    L, p = _prog()
    _, x = _v(L.pg_prog_input, p, n)
    _, sx = _v(L.pg_prog_scale, p, x, 3.0)
    _, y = _v(L.pg_prog_stencil, p, sx, 3, off, cf)
    _, m = _v(L.pg_prog_mul, p, y, sx)
    assert L.pg_prog_sum(p, m) == P.OK
    assert L.pg_prog_plan(p, ctypes.byref(sz)) == P.OK
    assert L.pg_prog_info(p, ctypes.byref(st)) == P.OK
    assert st.folded_ops == 0
    L.pg_prog_destroy(p)


def test_program_fusion_level_is_checked():
    L, p = _prog()
    assert L.pg_prog_fusion(p, 2) == P.EINVAL
    assert L.pg_prog_info(p, ctypes.byref(P.ProgStats())) == P.ESTATE
    L.pg_prog_destroy(p)
