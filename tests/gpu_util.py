"""Shared helpers for the GPU parity tests (no method arithmetic here)."""
import os
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_05231_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        raise RuntimeError("libnufftct.so missing on a GPU host: build it before running GPU tests")


def to_dev(a: np.ndarray, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.complex128)


def rel_l2(a, b) -> float:
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b) -> float:
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
