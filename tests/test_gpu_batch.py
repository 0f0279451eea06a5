"""Parity of the one-launch uneven-batch path with the per-instance oracle."""
import numpy as np
import pytest

import oracle
from paper_2507_13204_amd import inputs
from _helpers import TOL_F32, TOL_F64_F, TOL_F64_G, rel, srel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _batch(bt, dtype=torch.float64, **kw):
    from paper_2507_13204_amd import MeshBatch
    return (MeshBatch(bt.inst, to_dev(bt.conn), to_dev(bt.B, dtype), to_dev(bt.w, dtype), **kw),
            to_dev(bt.x, dtype))


def _check(bt, f, g, fbar=None, tol_f=TOL_F64_F, tol_g=TOL_F64_G):
    fs_ref, g_ref = oracle.mesh_batch_gradient(bt)
    if fbar is not None:
        g_ref = g_ref.copy()
        for i in range(bt.n_inst):
            nn, _, no, _ = bt.inst[i]
            g_ref[no:no + nn] = fbar[i] * oracle.mesh_gradient(*_inst_args(bt, i))[1]
    if f is not None:
        for a, b in zip(f, fs_ref):
            assert srel(a, b) <= tol_f
    assert rel(g, g_ref) <= tol_g


def _inst_args(bt, i):
    m = bt.instance(i)
    return m.n_nodes, m.conn, m.B, m.w, m.x


@pytest.mark.parametrize("block,tile", [(256, 1), (64, 2), (128, 4)])
@pytest.mark.parametrize("ckpt", ["recompute", "store"])
def test_batch_parity(block, tile, ckpt):
    bt = inputs.uneven_batch(12, seed=60, lo=3, hi=14)
    obj, x = _batch(bt, block=block, tile=tile, ckpt=ckpt)
    f, g = obj.gradient(x)
    _check(bt, f.cpu().numpy(), g.cpu().numpy())
    f2 = obj.objective(x).cpu().numpy()
    fbar = torch.linspace(-1.0, 2.0, bt.n_inst, dtype=torch.float64, device="cuda")
    g2 = obj.adjoint(x, fbar)
    _check(bt, f2, g2.cpu().numpy(), fbar=fbar.cpu().numpy())
    # per-instance results match one-instance plans
    from paper_2507_13204_amd import MeshObjective
    m = bt.instance(3)
    one = MeshObjective(to_dev(m.conn), to_dev(m.B), to_dev(m.w), m.n_nodes)
    f1 = one.objective(to_dev(m.x)).item()
    assert srel(f[3].item(), f1) <= 1e-14


def test_batch_f32_and_empty_instances():
    bt = inputs.uneven_batch(6, seed=61, lo=2, hi=9)
    obj, x = _batch(bt, torch.float32)
    b32 = bt.astype(np.float32)
    fs_ref, g_ref = oracle.mesh_batch_gradient(b32.astype(np.float64))
    for _ in range(3):  # the FP64 accumulation buffer is left zero by each call
        f, g = obj.gradient(x)
        assert rel(g.cpu().numpy(), g_ref) <= TOL_F32
        for a, b in zip(f.cpu().numpy(), fs_ref):
            assert srel(a, b) <= TOL_F32
    # an instance with no elements (side 1) gives f = 0 and grad = 0
    bt1 = inputs.uneven_batch(3, seed=62, sides=[4, 1, 3])
    obj, x = _batch(bt1)
    f, g = obj.gradient(x)
    assert f[1].item() == 0.0
    _check(bt1, f.cpu().numpy(), g.cpu().numpy())


def test_batch_full_size_graph_replay():
    """256 instances with sides log-uniform in [10, 100], one launch,
    captured once in a HIP graph and replayed."""
    bt = inputs.uneven_batch(256)
    obj, x = _batch(bt)
    fs_ref, g_ref = oracle.mesh_batch_gradient(bt)
    g = torch.empty_like(x)
    f = torch.empty(bt.n_inst, dtype=torch.float64, device="cuda")
    from paper_2507_13204_amd import pgrad as P
    import ctypes
    # eager reference
    f_e, g_e = obj.gradient(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        obj.gradient(x, out=g)  # warm-up on the capture stream
        with torch.cuda.graph(graph, stream=s):
            P.check(P.lib().pg_gradient(obj._plan, P._ptr(x), P._ptr(g), P._ptr(f),
                                        ctypes.c_void_p(s.cuda_stream)), "pg_gradient")
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        g.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _check(bt, f.cpu().numpy(), g.cpu().numpy())
        assert rel(g.cpu().numpy(), g_e.cpu().numpy()) <= 1e-13


@pytest.mark.parametrize("k", [2, 4, 5, 8])
def test_batch_of_random_meshes(k):
    """Instances with arbitrary connectivity (k = 5 takes the runtime-k kernel)."""
    meshes = [inputs.random_mesh(nn, ne, k, 90 + i) for i, (nn, ne) in
              enumerate([(40, 70), (7, 3), (300, 999), (1, 2), (64, 0), (500, 257)])]
    inst, no, eo = [], 0, 0
    for m in meshes:
        inst.append((m.n_nodes, m.n_elems, no, eo))
        no += m.n_nodes
        eo += m.n_elems
    bt = inputs.MeshBatch(np.array(inst, dtype=np.int64), k,
                          np.concatenate([m.conn for m in meshes]),
                          np.concatenate([m.B for m in meshes]),
                          np.concatenate([m.w for m in meshes]),
                          np.concatenate([m.x for m in meshes]), np.zeros(len(meshes)))
    obj, x = _batch(bt, block=128)
    f, g = obj.gradient(x)
    _check(bt, f.cpu().numpy(), g.cpu().numpy())
