"""Shared helpers of the test suite (comparison measures, device transfer)."""
import numpy as np

# Acceptance bars: FP64 primal rel <= 1e-12, gradient normwise rel <= 1e-10;
# FP32 <= 1e-5 against the oracle on the FP32-rounded inputs.
TOL_F64_F = 1e-12
TOL_F64_G = 1e-10
TOL_F32 = 1e-5


def rel(a, b) -> float:
    """Normwise relative error ||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def srel(a: float, b: float) -> float:
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


def to_dev(arr, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(arr))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def mesh_to_dev(m, dtype):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    return (to_dev(m.conn), to_dev(m.B, tdt), to_dev(m.w, tdt), to_dev(m.x, tdt))
