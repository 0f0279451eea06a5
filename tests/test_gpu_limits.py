"""The HIP mesh path at the edges of its index range (through the C ABI):
the largest incidence count (n_elems * k just under 2^31) and the largest node
index (n_nodes = 2^31 - 1), against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2507_13204_amd import inputs
from _helpers import TOL_F64_F, TOL_F64_G, rel, srel, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mesh_obj(conn, B, w, n_nodes, **kw):
    from paper_2507_13204_amd import MeshObjective
    return MeshObjective(to_dev(conn), to_dev(B), to_dev(w), n_nodes, **kw)


def test_largest_incidence_count():
    """k = 8, n_elems = (2^31 - 1) // 8: 2,147,483,640 incidences, the most a
    plan accepts.  Full-size f and gradient against the oracle (every entry)."""
    k = 8
    E = (2 ** 31 - 1) // k
    m = inputs.ring_mesh(E, k)
    assert m.conn.size == 2 ** 31 - 8 and int(m.conn.max()) == E - 1
    print(f"ring mesh: {E} elements, {m.conn.size} incidences", flush=True)
    obj = _mesh_obj(m.conn, m.B, m.w, m.n_nodes)
    x = to_dev(m.x)
    f, g = obj.gradient(x)
    f_obj = obj.objective(x).item()
    g = g.cpu().numpy()
    obj.close()
    del x
    torch.cuda.empty_cache()
    f_ref, g_ref = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
    assert srel(f.item(), f_ref) <= TOL_F64_F
    assert srel(f_obj, f_ref) <= TOL_F64_F
    assert rel(g, g_ref) <= TOL_F64_G


@pytest.mark.parametrize("adj", ["atomic", "gather", "tiled"])
def test_largest_node_index(adj):
    """n_nodes = 2^31 - 1 with elements on nodes at both ends of the range,
    the last node included.  The oracle runs on the touched nodes renumbered
    (relabelling nodes changes nothing else); every other gradient entry must
    be exactly zero."""
    N = 2 ** 31 - 1
    mm = inputs.wide_index_mesh(N, 4096, 8, span=1 << 16)
    print(f"wide-index mesh: {N} nodes, {mm.x_nodes.size} touched, {adj}", flush=True)
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    idx = torch.from_numpy(mm.x_nodes).cuda()
    x[idx] = to_dev(mm.x_vals)
    obj = _mesh_obj(mm.conn, mm.B, mm.w, N, adjoint=adj)
    f, g = obj.gradient(x)
    g_t = g[idx].cpu().numpy()
    nz = int(torch.count_nonzero(g).item())
    obj.close()
    del g, x
    torch.cuda.empty_cache()
    local = np.searchsorted(mm.x_nodes, mm.conn.astype(np.int64)).astype(np.int32)
    f_ref, g_ref = oracle.mesh_gradient(mm.x_nodes.size, local, mm.B, mm.w, mm.x_vals)
    assert srel(f.item(), f_ref) <= TOL_F64_F
    assert rel(g_t, g_ref) <= TOL_F64_G
    assert nz == int(np.count_nonzero(g_t))
