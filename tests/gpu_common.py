"""Shared helpers of the GPU parity tests: device transfer and case printing."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b)) if b.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / den)


def periodic_rel(a, b, L):
    worst = 0.0
    for d in range(3):
        diff = np.asarray(a[d], dtype=np.float64) - np.asarray(b[d], dtype=np.float64)
        diff = diff - L[d] * np.round(diff / L[d])
        if diff.size:
            worst = max(worst, float(np.max(np.abs(diff))) / L[d])
    return worst


def round32(a):
    """FP32 rounding of a host array, returned as FP64 (the values the FP32 kernels see)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)
