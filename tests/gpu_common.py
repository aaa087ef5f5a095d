"""Shared helpers of the GPU parity tests."""
import numpy as np


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def planar(hwc):
    """Oracle [h, w, C] -> library layout [C, h, w]."""
    return np.ascontiguousarray(np.moveaxis(hwc, -1, 0))


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU (run with -m 'not gpu' on CPU)"
