"""The paper's section 4 example on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
from _helpers import TOL_F32, TOL_F64_F, TOL_F64_G, rel, srel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)


@pytest.mark.parametrize("n", [1, 2, 3, 100, 255, 256, 257, 10_000, 16_384, 16_385, 1_000_003])
@pytest.mark.parametrize("adjoint", ["gather", "atomic"])
def test_laplace1d_parity(n, adjoint):
    from paper_2507_13204_amd import Laplace1D
    x, b = _inputs(n, n)
    lp = Laplace1D(n, adjoint=adjoint)
    f, gx, gb = lp.gradient(to_dev(x), to_dev(b))
    f_ref, gx_ref, gb_ref = oracle.laplace1d_gradient(x, b)
    assert srel(f.item(), f_ref) <= TOL_F64_F
    assert rel(gx.cpu().numpy(), gx_ref) <= TOL_F64_G
    assert rel(gb.cpu().numpy(), gb_ref) <= TOL_F64_G
    f_obj = lp.objective(to_dev(x), to_dev(b)).item()
    assert srel(f_obj, f_ref) <= TOL_F64_F
    if adjoint == "gather":  # same reduction order in the objective and the gradient
        assert f_obj == f.item()


@pytest.mark.parametrize("adjoint", ["gather", "atomic"])
def test_laplace1d_f32_accumulate_and_partial_outputs(adjoint):
    from paper_2507_13204_amd import Laplace1D
    n = 4097
    x, b = _inputs(n, 7)
    x32, b32 = x.astype(np.float32), b.astype(np.float32)
    lp = Laplace1D(n, dtype=torch.float32, adjoint=adjoint)
    f, gx, gb = lp.gradient(to_dev(x32), to_dev(b32))
    f_ref, gx_ref, gb_ref = oracle.laplace1d_gradient(x32.astype(np.float64), b32.astype(np.float64))
    assert srel(f.item(), f_ref) <= TOL_F32
    assert rel(gx.cpu().numpy(), gx_ref) <= TOL_F32 and rel(gb.cpu().numpy(), gb_ref) <= TOL_F32
    # accumulate: the shadow-argument convention of the generated code
    la = Laplace1D(n, adjoint=adjoint, accumulate=True)
    gx0 = torch.ones(n, dtype=torch.float64, device="cuda")
    gb0 = torch.full((n,), -2.0, dtype=torch.float64, device="cuda")
    _, gx1, gb1 = la.gradient(to_dev(x), to_dev(b), gx=gx0, gb=gb0)
    _, gxr, gbr = oracle.laplace1d_gradient(x, b)
    assert rel(gx1.cpu().numpy(), 1.0 + gxr) <= TOL_F64_G
    assert rel(gb1.cpu().numpy(), -2.0 + gbr) <= TOL_F64_G
    # only one of the two gradients
    l1 = Laplace1D(n, adjoint=adjoint)
    _, gxo, gbo = l1.gradient(to_dev(x), to_dev(b), want=("x",))
    assert gbo is None and rel(gxo.cpu().numpy(), gxr) <= TOL_F64_G


def test_laplace1d_errors():
    from paper_2507_13204_amd import Laplace1D
    from paper_2507_13204_amd.pgrad import EALIAS, EUNSUPPORTED, PgError
    lp = Laplace1D(64)
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    b = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(PgError) as ei:
        lp.gradient(x, b, gx=x)
    assert ei.value.code == EALIAS
    with pytest.raises(PgError) as ei:
        Laplace1D(8, adjoint="colour")
    assert ei.value.code == EUNSUPPORTED
    f, gx, gb = lp.gradient(x, b)
    assert f.item() == 0.0 and not torch.any(gx) and not torch.any(gb)


@pytest.mark.parametrize("adjoint", ["gather", "atomic"])
@pytest.mark.parametrize("n", [300, 16_384])
def test_laplace1d_in_a_graph(adjoint, n):
    """The one-launch form (the last workgroup sums the partials through a
    ticket it re-arms) captured in a HIP graph and replayed, with the outputs
    cleared by eager work in between; every replay matches the eager call."""
    from paper_2507_13204_amd import Laplace1D
    x, b = _inputs(n, 11)
    xd, bd = to_dev(x), to_dev(b)
    lp = Laplace1D(n, adjoint=adjoint)
    f_e, gx_e, gb_e = lp.gradient(xd, bd)
    gx, gb = torch.empty_like(xd), torch.empty_like(bd)
    f = torch.empty((), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        lp.gradient(xd, bd, gx=gx, gb=gb, f_out=f, stream=s)
        with torch.cuda.graph(graph, stream=s):
            lp.gradient(xd, bd, gx=gx, gb=gb, f_out=f, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    _, gx_ref, gb_ref = oracle.laplace1d_gradient(x, b)
    for _ in range(3):
        f.fill_(float("nan"))
        gx.zero_()
        gb.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert f.item() == f_e.item()
        assert rel(gx.cpu().numpy(), gx_ref) <= TOL_F64_G and rel(gb.cpu().numpy(), gb_ref) <= TOL_F64_G
        f_obj = lp.objective(xd, bd).item()  # the ticket is re-armed for eager calls too
        assert srel(f_obj, f_e.item()) <= 1e-15
