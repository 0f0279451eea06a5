"""Parity of the dense (team/vector) and batched dense (MFMA) paths."""
import math

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


# 16 columns of the 4096 x 1024 benchmark: both ends, every tile column
# boundary pair of one 128-wide tile, and spread samples.
FULL_COLS = [0, 1, 63, 64, 127, 128, 129, 255, 256, 511, 512, 700, 895, 1000, 1022, 1023]


@pytest.fixture(scope="module")
def bd_full():
    return inputs.batched_dense(4096, 1024)


def test_bdense_full_size_sampled_columns(bd_full):
    """A 4096 x 4096, X 4096 x 1024, FP64 MFMA: 16 gradient columns against the
    Dot2 oracle, f against the fast oracle."""
    b = bd_full
    obj, X = _bdense(b)
    f, G = obj.gradient(X)
    fc, Gc = oracle.bdense_columns(b.A, b.X, b.W, FULL_COLS)
    Gh = G.cpu().numpy()
    for t, c in enumerate(FULL_COLS):
        assert rel(Gh[:, c], Gc[:, t]) <= TOL_F64_G, c
    f_ref, _ = oracle.bdense_gradient_fast(b.A, b.X, b.W)
    assert srel(f.item(), f_ref) <= TOL_F64_F


def test_bdense_full_size_f32(bd_full):
    """FP32 storage on the FP32 matrix cores at the benchmark shape: f and 16
    gradient columns against the Dot2 oracle on the FP32-rounded inputs
    (1e-5); the error against the FP64-input oracle is reported."""
    b = bd_full
    obj, X = _bdense(b, torch.float32)
    f, G = obj.gradient(X)
    A32, X32, W32 = (a.astype(np.float32).astype(np.float64) for a in (b.A, b.X, b.W))
    fc, Gc = oracle.bdense_columns(A32, X32, W32, FULL_COLS)
    Gh = G.cpu().numpy().astype(np.float64)
    errs = [rel(Gh[:, c], Gc[:, t]) for t, c in enumerate(FULL_COLS)]
    assert max(errs) <= TOL_F32, max(errs)
    f_ref, _ = oracle.bdense_gradient_fast(A32, X32, W32)
    assert srel(f.item(), f_ref) <= TOL_F32
    f64_ref, _ = oracle.bdense_gradient_fast(b.A, b.X, b.W)
    _, Gc64 = oracle.bdense_columns(b.A, b.X, b.W, FULL_COLS)
    e64 = max(rel(Gh[:, c], Gc64[:, t]) for t, c in enumerate(FULL_COLS))
    print(f"bdense FP32 4096x4096x1024: gradient columns {max(errs):.2e} (rounded inputs), "
          f"{e64:.2e} (FP64 inputs); f {srel(f.item(), f_ref):.2e} / {srel(f.item(), f64_ref):.2e}")
    assert e64 <= 1e-4


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_bdense_fn_full_size_fd_16_directions(bd_full, dtype):
    """The autograd form at 4096 x 1024: central differences of the GPU
    objective on 16 random unit-norm directions against <G, Xp - Xm>.
    FP64: h = 1e-4, 1e-6 relative.  FP32: the perturbed points are rounded
    to FP32, so the difference is taken against the exact step Xp - Xm.
    Each FP32 evaluation of f carries rounding noise that does not shrink
    with h: the products Y = A X are accurate to about 2^-24 |Y| per entry
    (|Y| ~ 0.6), and the 4M errors add like a random walk in
    f = sum W psi(Y), about 2048 * 6e-8 * 0.6 = 7e-5 per evaluation (1.5e-4
    was seen in f(Xp) - f(Xm) at h = 1e-2, where the slope is only 0.0125).
    So h = 1: the slope is about 1.2, the noise about 1e-4 of it, and the
    third-order term about 2e-7 of it ((A D) entries are ~5e-4); bar 1e-3."""
    from paper_2507_13204_amd import BatchedDense, BatchedDenseFn
    b = bd_full
    obj = BatchedDense(to_dev(b.A, dtype), to_dev(b.W, dtype))
    X = to_dev(b.X, dtype).requires_grad_(True)
    BatchedDenseFn.apply(X, obj).backward()
    G = X.grad.double()
    h, tol = (1e-4, 1e-6) if dtype == torch.float64 else (1.0, 1e-3)
    with torch.no_grad():
        for D in inputs.fd_directions(b.X.shape, 16, seed=33):
            Dt = to_dev(D)
            Xp = (X.detach().double() + h * Dt).to(dtype)
            Xm = (X.detach().double() - h * Dt).to(dtype)
            fp = obj.objective(Xp).item()
            fm = obj.objective(Xm).item()
            slope = (G * (Xp.double() - Xm.double())).sum().item()
            assert abs((fp - fm) - slope) <= tol * max(1.0, abs(slope)), (fp - fm, slope)


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
