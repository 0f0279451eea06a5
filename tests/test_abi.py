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
    assert L.pg_version() == 1


def test_default_options():
    o = P.lib().pg_default_options()
    assert (o.adjoint, o.ckpt, o.block, o.tile, o.accumulate, o.scatter) == (0, 0, 0, 0, 0, 0)


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
    st, plan, ws = plan_mesh(n_nodes=1000, n_elems=900, k=8)
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
])
def test_mesh_plan_argument_errors(kw, code):
    if kw.get("opts") == "bad_adjoint":
        kw["opts"] = P.make_options(adjoint=9)
    elif kw.get("opts") == "bad_block":
        kw["opts"] = P.make_options(block=100)
    elif kw.get("opts") == "bad_tile":
        kw["opts"] = P.make_options(tile=3)
    st, plan, _ = plan_mesh(**kw)
    assert st == code
    assert not plan.value
    assert len(P.lib().pg_last_error()) > 0


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
