"""Helpers shared by the GPU tests (device selection, tensor transfer)."""
import os

import numpy as np
import pytest


def device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_00538_amd as lib
    lib.load_library()        # fails loudly if the HIP library is missing
    return torch.device("cuda:0")


def to_dev(a, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
