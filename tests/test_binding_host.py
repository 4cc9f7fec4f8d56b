"""The torch binding refuses buffers the kernels could not address (host tensors, workspaces of the
wrong type) on the host, before any library call: no GPU is needed for these checks."""
import os

import pytest
import torch

from paper_2602_20870_amd import _lib


@pytest.fixture(scope="module")
def ops():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libfgfrft.so not built")
    from paper_2602_20870_amd import ops as o
    return o


def test_host_tensors_are_refused(ops):
    Q = torch.zeros((2, 8, 8), dtype=torch.complex64)
    X = torch.zeros((2, 8, 4), dtype=torch.float32)
    with pytest.raises(ValueError, match="cuda"):
        ops.apply_operator(Q, X)
    V = torch.zeros((8, 8), dtype=torch.complex128)
    with pytest.raises(ValueError, match="cuda"):
        ops.gfrft_exact(V, V, torch.zeros(8, dtype=torch.float64), 0.5)
    cuda0 = torch.device("cuda", 0)
    with pytest.raises(ValueError, match="cuda"):
        ops._on_device(cuda0, out=torch.zeros(4))
    ops._on_device(cuda0, out=None)          # absent buffers are skipped


def test_caller_workspace_must_be_device_bytes(ops):
    cuda0 = torch.device("cuda", 0)
    with pytest.raises(ValueError, match="cuda"):
        ops._caller_ws(torch.zeros(1024, dtype=torch.uint8), 256, cuda0)


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback path: without the built library the first call raises."""
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(os.path.dirname(_lib.LIB_PATH), "no_such_libfgfrft.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()
