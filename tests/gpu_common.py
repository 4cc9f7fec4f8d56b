"""Shared helpers for the GPU parity tests (inputs from synth, expectations from oracle)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Parity bar for the FP32 path: relative Frobenius error per order against the FP64 oracle.
TOL_FP32 = 1e-5
# BF16 hi/lo stack: each real value keeps ~16 bits (|x - hi - lo| <= 2^-16 |x|) and the
# lo*lo product is dropped; measured errors sit near 3e-6 to 1e-5, the stated bar is 5e-5.
TOL_BF16X2 = 5e-5


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_fro(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def announce(msg):
    print(f"[case] {msg}", flush=True)
