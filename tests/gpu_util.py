"""Helpers shared by the GPU tests (inputs to device, results to host)."""
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1211_5481_amd import _lib
    _lib.lib()  # raises if libgame.so is missing: no silent fallback
    return torch


def dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def announce(msg: str):
    """Name the case before a GPU step, so a crash report points at it."""
    sys.stdout.write(f"[gpu-case] {msg}\n")
    sys.stdout.flush()
