"""Helpers shared by the GPU tests: device availability and the parity metric."""
import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def rel(a, b):
    """Normwise relative difference ||a - b||_2 / ||b||_2."""
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
