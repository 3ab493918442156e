"""Helpers shared by the GPU tests (marshalling and tolerances only)."""
import numpy as np


def device():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device())


def header(msg):
    """Name the case before each GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
