"""Per-call tapes, the refusal of a tape recorded from another x, the
checkpoint choice by memory and the autograd policies, against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2507_13204_amd import inputs
from _helpers import TOL_F32, TOL_F64_F, TOL_F64_G, rel, srel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _mesh_obj(m, **kw):
    from paper_2507_13204_amd import MeshObjective
    return MeshObjective(to_dev(m.conn), to_dev(m.B), to_dev(m.w), m.n_nodes, **kw)


def _other_x(n, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


@pytest.mark.parametrize("policy", ["gradient", "store", "recompute"])
@pytest.mark.parametrize("adj", ["atomic", "gather", "tiled", "colour"])
@pytest.mark.parametrize("ckpt", ["store", "recompute"])
def test_meshfn_two_forwards_then_one_backward(policy, adj, ckpt):
    """f1 = f(x1), f2 = f(x2) on one plan, then one backward of f1 + 2 f2:
    each forward keeps its own saved state, so both gradients are exact."""
    from paper_2507_13204_amd import MeshFn
    m = inputs.hex_mesh(12, seed=80)
    obj = _mesh_obj(m, adjoint=adj, ckpt=ckpt, autograd=policy)
    assert obj.autograd_policy == policy
    x2h = _other_x(m.n_nodes, 81)
    x1 = to_dev(m.x).requires_grad_(True)
    x2 = to_dev(x2h).requires_grad_(True)
    f1 = MeshFn.apply(x1, obj)
    f2 = MeshFn.apply(x2, obj)
    (f1 + 2.0 * f2).backward()
    f1r, g1 = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    f2r, g2 = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, x2h)
    assert srel(f1.item(), f1r) <= TOL_F64_F and srel(f2.item(), f2r) <= TOL_F64_F
    assert rel(x1.grad.cpu().numpy(), g1) <= TOL_F64_G
    assert rel(x2.grad.cpu().numpy(), 2.0 * g2) <= TOL_F64_G


def test_meshfn_same_tensor_changed_in_place_between_forwards():
    """The saved state of a forward is its own: changing x after the first
    forward (torch bumps its version) does not leak into the first term."""
    from paper_2507_13204_amd import MeshFn
    m = inputs.hex_mesh(10, seed=82)
    for policy in ("gradient", "store"):
        obj = _mesh_obj(m, autograd=policy)
        xa = to_dev(m.x).requires_grad_(True)
        f1 = MeshFn.apply(xa * 1.0, obj)
        f2 = MeshFn.apply(xa * 0.5, obj)
        (f1 - f2).backward()
        _, g1 = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
        _, g2 = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, 0.5 * m.x)
        assert rel(xa.grad.cpu().numpy(), g1 - 0.5 * g2) <= TOL_F64_G


@pytest.mark.parametrize("policy", ["gradient", "store", "recompute"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_dense_fn_two_forwards(policy, dtype):
    from paper_2507_13204_amd import BatchedDense, BatchedDenseFn
    b = inputs.batched_dense(192, 80, seed=83)
    obj = BatchedDense(to_dev(b.A, dtype), to_dev(b.W, dtype), autograd=policy)
    X2h = np.random.default_rng(84).uniform(-1, 1, b.X.shape)
    X1 = to_dev(b.X, dtype).requires_grad_(True)
    X2 = to_dev(X2h, dtype).requires_grad_(True)
    (BatchedDenseFn.apply(X1, obj) + 2.0 * BatchedDenseFn.apply(X2, obj)).backward()
    if dtype == torch.float32:
        A, W = (a.astype(np.float32).astype(np.float64) for a in (b.A, b.W))
        X1h = b.X.astype(np.float32).astype(np.float64)
        X2h = X2h.astype(np.float32).astype(np.float64)
        tol = TOL_F32
    else:
        A, W, X1h, tol = b.A, b.W, b.X, TOL_F64_G
    _, G1 = oracle.bdense_gradient_fast(A, X1h, W)
    _, G2 = oracle.bdense_gradient_fast(A, X2h, W)
    assert rel(X1.grad.cpu().numpy(), G1) <= tol
    assert rel(X2.grad.cpu().numpy(), 2.0 * G2) <= tol


@pytest.mark.parametrize("policy", ["store", "recompute"])
def test_mesh_batch_fn_two_forwards(policy):
    from paper_2507_13204_amd import MeshBatch, MeshBatchFn
    bt = inputs.uneven_batch(6, seed=85, lo=3, hi=9)
    ob = MeshBatch(bt.inst, to_dev(bt.conn), to_dev(bt.B), to_dev(bt.w), autograd=policy)
    assert ob.autograd_policy == policy
    x2h = _other_x(bt.x.shape[0], 86)
    x1 = to_dev(bt.x).requires_grad_(True)
    x2 = to_dev(x2h).requires_grad_(True)
    wts = torch.arange(1, bt.n_inst + 1, dtype=torch.float64, device="cuda")
    ((MeshBatchFn.apply(x1, ob) * wts).sum() + 2.0 * MeshBatchFn.apply(x2, ob).sum()).backward()
    _, g1 = oracle.mesh_batch_gradient(bt)
    bt2 = inputs.uneven_batch(6, seed=85, lo=3, hi=9)
    bt2.x[:] = x2h
    _, g2 = oracle.mesh_batch_gradient(bt2)
    want1 = g1.copy()
    for i in range(bt.n_inst):
        nn, _, no, _ = bt.inst[i]
        want1[no:no + nn] *= (i + 1)
    assert rel(x1.grad.cpu().numpy(), want1) <= TOL_F64_G
    assert rel(x2.grad.cpu().numpy(), 2.0 * g2) <= TOL_F64_G


# ------------------------------------------------- the workspace's own tape

@pytest.mark.parametrize("name,mk", [("hex14", lambda: inputs.hex_mesh(14, seed=87)),
                                     ("hex40", lambda: inputs.hex_mesh(40, seed=88))])
def test_stored_tape_of_another_x_is_refused(name, mk):
    """ckpt = store: pg_adjoint reads the workspace's tape only for the x it
    was recorded from; any other x is PG_ESTATE (nothing enqueued).  hex14 is
    a one-launch plan, hex40 the multi-launch path."""
    from paper_2507_13204_amd.pgrad import ESTATE, PgError
    m = mk()
    obj = _mesh_obj(m, ckpt="store")
    x1 = to_dev(m.x)
    x2 = to_dev(_other_x(m.n_nodes, 89))
    fbar = torch.ones(1, dtype=torch.float64, device="cuda")
    obj.objective(x1)
    with pytest.raises(PgError) as ei:
        obj.adjoint(x2, fbar)
    assert ei.value.code == ESTATE
    g = obj.adjoint(x1, fbar)
    _, g_ref = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    assert rel(g.cpu().numpy(), g_ref) <= TOL_F64_G


def test_batched_dense_gradient_invalidates_the_stored_v():
    """objective(X1), gradient(X2), adjoint(X1): the gradient overwrote V, so
    the adjoint is refused instead of returning the gradient at X2."""
    from paper_2507_13204_amd import BatchedDense
    from paper_2507_13204_amd.pgrad import ESTATE, PgError
    b = inputs.batched_dense(128, 64, seed=90)
    obj = BatchedDense(to_dev(b.A), to_dev(b.W), ckpt="store")
    X1 = to_dev(b.X)
    X2 = to_dev(np.random.default_rng(91).uniform(-1, 1, b.X.shape))
    fbar = torch.ones(1, dtype=torch.float64, device="cuda")
    obj.objective(X1)
    obj.gradient(X2)
    with pytest.raises(PgError) as ei:
        obj.adjoint(X1, fbar)
    assert ei.value.code == ESTATE
    with pytest.raises(PgError):
        obj.adjoint(X2, fbar)  # a gradient records no tape
    obj.objective(X1)
    G = obj.adjoint(X1, fbar)
    _, G_ref = oracle.bdense_gradient_fast(b.A, b.X, b.W)
    assert rel(G.cpu().numpy(), G_ref) <= TOL_F64_G


def test_batch_stored_tape_of_another_x_is_refused():
    from paper_2507_13204_amd import MeshBatch
    from paper_2507_13204_amd.pgrad import ESTATE, PgError
    bt = inputs.uneven_batch(4, seed=92, lo=3, hi=7)
    ob = MeshBatch(bt.inst, to_dev(bt.conn), to_dev(bt.B), to_dev(bt.w), ckpt="store")
    x1 = to_dev(bt.x)
    x2 = to_dev(_other_x(bt.x.shape[0], 93))
    fbar = torch.ones(bt.n_inst, dtype=torch.float64, device="cuda")
    ob.objective(x1)
    with pytest.raises(PgError) as ei:
        ob.adjoint(x2, fbar)
    assert ei.value.code == ESTATE
    _, g_ref = oracle.mesh_batch_gradient(bt)
    assert rel(ob.adjoint(x1, fbar).cpu().numpy(), g_ref) <= TOL_F64_G


# --------------------------------------------------------- per-call tapes

@pytest.mark.parametrize("name,mk,kw", [
    ("hex14_onelaunch", lambda: inputs.hex_mesh(14, seed=94), {}),
    ("hex30_atomic", lambda: inputs.hex_mesh(30, seed=95), {"onepass": False}),
    ("hex30_tiled", lambda: inputs.hex_mesh(30, seed=95), {"adjoint": "tiled"}),
    ("hex30_colour", lambda: inputs.hex_mesh(30, seed=95), {"adjoint": "colour"}),
    ("rand_k5", lambda: inputs.random_mesh(700, 999, 5, 9), {"adjoint": "gather"}),
])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_per_call_tape_matches_the_oracle(name, mk, kw, dtype):
    m = mk()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    from paper_2507_13204_amd import MeshObjective
    obj = MeshObjective(to_dev(m.conn), to_dev(m.B, tdt), to_dev(m.w, tdt), m.n_nodes, **kw)
    assert obj.tape_bytes() == 8 * m.n_elems
    xs = [m.x, _other_x(m.n_nodes, 96)]
    tapes = [obj.new_tape("cuda") for _ in xs]
    fs = [obj.objective_tape(to_dev(x, tdt), t) for x, t in zip(xs, tapes)]
    fbar = torch.tensor([-1.25], dtype=torch.float64, device="cuda")
    gs = [obj.adjoint_tape(fbar, t, to_dev(x, tdt)) for x, t in zip(xs, tapes)]
    mm = m.astype(np.float32) if dtype == "f32" else m
    for x, f, g in zip(xs, fs, gs):
        xr = x.astype(np.float32).astype(np.float64) if dtype == "f32" else x
        f_ref, g_ref = oracle.mesh_gradient(m.n_nodes, m.conn, mm.B.astype(np.float64),
                                            mm.w.astype(np.float64), xr, -1.25)
        ftol, gtol = (TOL_F64_F, TOL_F64_G) if dtype == "f64" else (TOL_F32, TOL_F32)
        assert srel(f.item(), oracle.mesh_objective(m.n_nodes, m.conn, mm.B.astype(np.float64),
                                                    mm.w.astype(np.float64), xr)) <= ftol
        assert rel(g.cpu().numpy(), g_ref) <= gtol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_dense_per_call_tape(dtype):
    from paper_2507_13204_amd import BatchedDense
    b = inputs.batched_dense(160, 48, seed=97)
    obj = BatchedDense(to_dev(b.A, dtype), to_dev(b.W, dtype), ckpt="recompute")
    assert obj.tape_bytes() == 160 * 48 * (8 if dtype == torch.float64 else 4)
    X = to_dev(b.X, dtype)
    tape = obj.new_tape("cuda")
    f = obj.objective_tape(X, tape)
    fbar = torch.tensor([0.75], dtype=torch.float64, device="cuda")
    G = obj.adjoint_tape(fbar, tape, X)
    if dtype == torch.float32:
        A, Xh, W = (a.astype(np.float32).astype(np.float64) for a in (b.A, b.X, b.W))
        tf, tg = TOL_F32, TOL_F32
    else:
        A, Xh, W, tf, tg = b.A, b.X, b.W, TOL_F64_F, TOL_F64_G
    f_ref, G_ref = oracle.bdense_gradient_fast(A, Xh, W, 0.75)
    assert srel(f.item(), oracle.bdense_gradient_fast(A, Xh, W)[0]) <= tf
    assert rel(G.cpu().numpy(), G_ref) <= tg


# ----------------------------------------------- checkpoint chosen by memory

@pytest.mark.parametrize("budget,want", [(0, "store"), (1, "recompute")])
def test_ckpt_auto_branches_match_the_oracle(budget, want):
    """ckpt = auto stores u_e when the tape fits the budget (0: a quarter of
    the free device memory, plenty here) and recomputes it otherwise; both
    give the oracle's gradient through objective + adjoint."""
    from paper_2507_13204_amd.pgrad import RECOMPUTE, STORE
    m = inputs.hex_mesh(33, seed=98)
    obj = _mesh_obj(m, ckpt="auto", tape_budget=budget)
    info = obj.info()
    assert info["ckpt"] == {"store": STORE, "recompute": RECOMPUTE}[want]
    assert info["tape_budget"] > 0 and info["tape_bytes"] == 8 * m.n_elems
    x = to_dev(m.x)
    obj.objective(x)
    fbar = torch.ones(1, dtype=torch.float64, device="cuda")
    g = obj.adjoint(x, fbar)
    _, g_ref = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    assert rel(g.cpu().numpy(), g_ref) <= TOL_F64_G


def test_autograd_auto_policy_follows_the_budget():
    """autograd = auto keeps the gradient if x's bytes fit the budget, else
    u_e on a tape if that fits, else nothing."""
    from paper_2507_13204_amd import MeshFn
    m = inputs.hex_mesh(12, seed=99)  # 1728 nodes, 1331 elements
    cases = [(1 << 30, "gradient"), (8 * 1331, "store"), (8 * 1331 - 1, "recompute")]
    _, g_ref = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    for budget, want in cases:
        obj = _mesh_obj(m, autograd="auto", autograd_budget=budget)
        assert obj.autograd_policy == want, (budget, obj.autograd_policy)
        x = to_dev(m.x).requires_grad_(True)
        MeshFn.apply(x, obj).backward()
        assert rel(x.grad.cpu().numpy(), g_ref) <= TOL_F64_G


def test_scale_rounds_once():
    from paper_2507_13204_amd import pgrad
    x = torch.linspace(-3, 3, 100_003, dtype=torch.float64, device="cuda")
    a = torch.tensor([-0.3], dtype=torch.float64, device="cuda")
    assert torch.equal(pgrad.scale(a, x), x * -0.3)
    x32 = x.float()
    want = (x32.double() * -0.3).float()
    y = pgrad.scale(a, x32)
    assert torch.equal(y, want)
    pgrad.scale(a, x32, out=x32)  # in place
    assert torch.equal(x32, want)
