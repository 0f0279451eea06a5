"""Parity of the dense (team/vector) and batched dense (MFMA) paths."""
import numpy as np
import pytest

import oracle
from paper_2507_13204_amd import inputs
from _helpers import TOL_F32, TOL_F64_F, TOL_F64_G, rel, srel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dense(d, dtype=torch.float64):
    from paper_2507_13204_amd import DenseObjective
    return DenseObjective(to_dev(d.A, dtype), to_dev(d.w, dtype)), to_dev(d.x, dtype)


@pytest.mark.parametrize("rows,cols", [(1, 1), (3, 7), (200, 300), (1000, 1024), (517, 2050),
                                       (64, 16384), (33, 16386), (20, 20001)])
def test_dense_parity_f64(rows, cols):
    d = inputs.dense(cols, seed=20 + rows, rows=rows)
    obj, x = _dense(d)
    f, g = obj.gradient(x)
    f_ref, g_ref = oracle.dense_gradient(d.A, d.x, d.w)
    assert srel(f.item(), f_ref) <= TOL_F64_F
    assert rel(g.cpu().numpy(), g_ref) <= TOL_F64_G
    assert srel(obj.objective(x).item(), f_ref) <= TOL_F64_F


def test_dense_parity_f32_and_seed():
    d = inputs.dense(3000, seed=31, rows=1500)
    obj, x = _dense(d, torch.float32)
    f, g = obj.gradient(x)
    A32, x32, w32 = (a.astype(np.float32).astype(np.float64) for a in (d.A, d.x, d.w))
    f_ref, g_ref = oracle.dense_gradient(A32, x32, w32)
    assert srel(f.item(), f_ref) <= TOL_F32 and rel(g.cpu().numpy(), g_ref) <= TOL_F32
    obj64, x64 = _dense(d)
    fbar = torch.tensor([2.5], dtype=torch.float64, device="cuda")
    g2 = obj64.adjoint(x64, fbar)
    _, g_ref2 = oracle.dense_gradient(d.A, d.x, d.w, 2.5)
    assert rel(g2.cpu().numpy(), g_ref2) <= TOL_F64_G


def test_dense_full_size():
    """A 10,000 x 10,000 with entries N(0, 1/n): the row-reduction workload."""
    d = inputs.dense(10_000)
    obj, x = _dense(d)
    f, g = obj.gradient(x)
    f_ref, g_ref = oracle.dense_gradient(d.A, d.x, d.w)
    assert srel(f.item(), f_ref) <= TOL_F64_F
    assert rel(g.cpu().numpy(), g_ref) <= TOL_F64_G
    fs = [obj.gradient(x)[1] for _ in range(2)]
    assert torch.equal(fs[0], fs[1])  # fixed-order column sums


def _bdense(b, dtype=torch.float64, ckpt="store"):
    from paper_2507_13204_amd import BatchedDense
    return BatchedDense(to_dev(b.A, dtype), to_dev(b.W, dtype), ckpt=ckpt), to_dev(b.X, dtype)


@pytest.mark.parametrize("m,n", [(1, 1), (16, 16), (128, 128), (200, 70), (257, 129), (512, 384)])
@pytest.mark.parametrize("ckpt", ["store", "recompute"])
def test_bdense_parity_f64(m, n, ckpt):
    b = inputs.batched_dense(m, n, seed=40 + m)
    obj, X = _bdense(b, ckpt=ckpt)
    f, G = obj.gradient(X)
    f_ref, G_ref = oracle.bdense_gradient_fast(b.A, b.X, b.W)
    assert srel(f.item(), f_ref) <= TOL_F64_F
    assert rel(G.cpu().numpy(), G_ref) <= TOL_F64_G
    f2 = obj.objective(X)
    fbar = torch.tensor([0.5], dtype=torch.float64, device="cuda")
    G2 = obj.adjoint(X, fbar)
    assert srel(f2.item(), f_ref) <= TOL_F64_F
    assert rel(G2.cpu().numpy(), 0.5 * G_ref) <= TOL_F64_G


@pytest.mark.parametrize("m,n", [(128, 64), (300, 200)])
def test_bdense_parity_f32(m, n):
    b = inputs.batched_dense(m, n, seed=50 + m)
    obj, X = _bdense(b, torch.float32)
    f, G = obj.gradient(X)
    A32, X32, W32 = (a.astype(np.float32).astype(np.float64) for a in (b.A, b.X, b.W))
    f_ref, G_ref = oracle.bdense_gradient_fast(A32, X32, W32)
    # FP32 MFMA accumulates inside the instruction in FP32
    assert srel(f.item(), f_ref) <= TOL_F32 and rel(G.cpu().numpy(), G_ref) <= TOL_F32


def test_bdense_full_size_sampled_columns():
    """A 4096 x 4096, X 4096 x 1024: sampled columns against the Dot2 oracle."""
    b = inputs.batched_dense(4096, 1024)
    obj, X = _bdense(b)
    f, G = obj.gradient(X)
    cols = [0, 1, 511, 1000, 1023]
    fc, Gc = oracle.bdense_columns(b.A, b.X, b.W, cols)
    Gh = G.cpu().numpy()
    for t, c in enumerate(cols):
        assert rel(Gh[:, c], Gc[:, t]) <= TOL_F64_G
    f_ref, _ = oracle.bdense_gradient_fast(b.A, b.X, b.W)
    assert srel(f.item(), f_ref) <= TOL_F64_F


def test_bdense_misaligned_operand_takes_the_scalar_path():
    """X at an 8-byte offset: the vector loads are not used, results still match."""
    b = inputs.batched_dense(256, 128, seed=57)
    obj, X = _bdense(b)
    big = torch.empty(X.numel() + 1, dtype=torch.float64, device="cuda")
    Xm = big[1:].view(X.shape)
    Xm.copy_(X)
    assert Xm.data_ptr() % 16 == 8
    f, G = obj.gradient(Xm)
    f_ref, G_ref = oracle.bdense_gradient_fast(b.A, b.X, b.W)
    assert srel(f.item(), f_ref) <= TOL_F64_F
    assert rel(G.cpu().numpy(), G_ref) <= TOL_F64_G
