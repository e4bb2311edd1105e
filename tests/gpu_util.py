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


def accumulation_bound(Phi, G, ref, t, task, M):
    """Worst-case float32 error of each chromosome's MSE when the rounded
    basis values and genes are exact on both sides (the 16-bit forms against
    the oracle on their stored inputs).  z is accumulated from M exact
    products in float32: |dz| <= g S with g = M 2^-24 and S = sum_m |Phi G|
    (plus 2^-24 |z| for adding a bias gene).
    Classification: the sigmoid has slope at most 1/4; exp, add and
    reciprocal round q by at most 3 2^-24 relative, and the rounding of the
    exponent z log2 e moves it by at most |z| 2^-24 relative; regression:
    dq = dz.  Then d(q^2) <= 2 |q| dq + dq^2, averaged over the patterns, plus
    32 2^-24 relative for the float32 sum of a 32-row unit."""
    gam = M * 2.0 ** -24
    z = ref["z"]
    dz = gam * (np.abs(Phi) @ np.abs(G[:, :M]).T) + 2.0 ** -24 * np.abs(z)  # + a bias gene's add
    if task == "classification":
        q = np.abs((t >= 0.5)[:, None] - 1.0 / (1.0 + np.exp(-z)))
        dq = dz / 4.0 + (3.0 + np.abs(z)) * 2.0 ** -24 * q
    else:
        q = np.abs(t[:, None] - z)
        dq = dz
    return np.mean(2.0 * q * dq + dq * dq, axis=0) + 32 * 2.0 ** -24 * ref["mse"]
