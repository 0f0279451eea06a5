"""torch.autograd.Function forms: backward seeded with grad_output."""
import numpy as np
import pytest

import oracle
from paper_2507_13204_amd import inputs
from _helpers import TOL_F64_G, rel, srel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("policy", ["gradient", "store", "recompute"])
@pytest.mark.parametrize("adj", ["atomic", "gather"])
def test_meshfn_backward_matches_oracle_and_fd(policy, adj):
    from paper_2507_13204_amd import MeshFn, MeshObjective
    m = inputs.hex_mesh(12, seed=70)
    obj = MeshObjective(to_dev(m.conn), to_dev(m.B), to_dev(m.w), m.n_nodes, adjoint=adj,
                        autograd=policy)
    x = to_dev(m.x).requires_grad_(True)
    f = MeshFn.apply(x, obj)
    (3.0 * f).backward()
    _, g_ref = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    assert rel(x.grad.cpu().numpy(), 3.0 * g_ref) <= TOL_F64_G
    # central finite differences through the forward kernel, 16 directions
    g = x.grad.cpu().numpy() / 3.0
    for d in inputs.fd_directions((m.n_nodes,), 16, seed=33):
        h = 1e-5
        dt = to_dev(d)
        fp = obj.objective(x.detach() + h * dt).item()
        fm = obj.objective(x.detach() - h * dt).item()
        assert abs((fp - fm) / (2 * h) - g @ d) <= 1e-6 * max(1.0, abs(g @ d))


def test_batched_dense_fn_fd_16_directions():
    from paper_2507_13204_amd import BatchedDense, BatchedDenseFn
    b = inputs.batched_dense(256, 96, seed=71)
    obj = BatchedDense(to_dev(b.A), to_dev(b.W), ckpt="store")
    X = to_dev(b.X).requires_grad_(True)
    f = BatchedDenseFn.apply(X, obj)
    f.backward()
    G = X.grad.cpu().numpy()
    _, G_ref = oracle.bdense_gradient_fast(b.A, b.X, b.W)
    assert rel(G, G_ref) <= TOL_F64_G
    for D in inputs.fd_directions(b.X.shape, 16, seed=33):
        h = 1e-5
        Dt = to_dev(D)
        fp = obj.objective(X.detach() + h * Dt).item()
        fm = obj.objective(X.detach() - h * Dt).item()
        assert abs((fp - fm) / (2 * h) - (G * D).sum()) <= 1e-6 * max(1.0, abs((G * D).sum()))


def test_dense_and_batch_fns():
    from paper_2507_13204_amd import DenseFn, DenseObjective, MeshBatch, MeshBatchFn
    d = inputs.dense(500, seed=72, rows=300)
    obj = DenseObjective(to_dev(d.A), to_dev(d.w))
    x = to_dev(d.x).requires_grad_(True)
    DenseFn.apply(x, obj).backward()
    _, g_ref = oracle.dense_gradient(d.A, d.x, d.w)
    assert rel(x.grad.cpu().numpy(), g_ref) <= TOL_F64_G
    bt = inputs.uneven_batch(5, seed=73, lo=3, hi=8)
    ob = MeshBatch(bt.inst, to_dev(bt.conn), to_dev(bt.B), to_dev(bt.w), ckpt="store")
    xb = to_dev(bt.x).requires_grad_(True)
    fs = MeshBatchFn.apply(xb, ob)
    wts = torch.arange(1, bt.n_inst + 1, dtype=torch.float64, device="cuda")
    (fs * wts).sum().backward()
    _, g_all = oracle.mesh_batch_gradient(bt)
    want = g_all.copy()
    for i in range(bt.n_inst):
        nn, _, no, _ = bt.inst[i]
        want[no:no + nn] *= (i + 1)
    assert rel(xb.grad.cpu().numpy(), want) <= TOL_F64_G
