"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import sys

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def announce(msg):
    """Print what the next GPU step is, flushed, so a failing run names it."""
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


def normwise(a, b):
    """||a - b||_inf / ||b||_inf (0 when both are zero)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b)) if b.size else 0.0
    num = np.max(np.abs(a - b)) if b.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den


def rel(a, b):
    if b == 0:
        return abs(a)
    return abs(a - b) / abs(b)
