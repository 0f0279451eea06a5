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


@pytest.mark.parametrize("n", [1, 2, 3, 100, 255, 256, 257, 10_000, 1_000_003])
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
    assert srel(lp.objective(to_dev(x), to_dev(b)).item(), f_ref) <= TOL_F64_F


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
