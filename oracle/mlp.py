"""Fitness-surrogate MLP -- oracle side, test infrastructure only.

A two-hidden-layer perceptron maps a chromosome g (L genes) to a score
y_hat = w3 . h2 + b3,  h2 = gelu(W2 h1 + b2),  h1 = gelu(W1 g + b1),
with the exact GELU gelu(a) = a Phi(a) = a (1 + erf(a / sqrt 2)) / 2.  It is
trained online to predict the standardised log MSE of chromosomes the GA has
evaluated exactly (loss: mean squared error over a minibatch), with Adam
(Kingma and Ba, ICLR 2015).  Plain float64 numpy; each function follows the
definition directly.

Initialisation: He-uniform (bound sqrt(6 / fan_in)) from Philox4x32-10 block
(layer, row, col, MLP_INIT) word 0 as u = ((w >> 8) + 1/2) 2^-24, weight =
bound (2u - 1); biases zero.  Minibatch draw i of training step s uses
w = word 0 of block (s, i, 0, MINIBATCH): most rows are uniform over the
replay buffer, a set fraction over the latest generation's evaluations
(``minibatch_slots``).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .philox import philox4x32_10

TAG_MLP_INIT = 7
TAG_MINIBATCH = 8


def gelu(a):
    a = np.asarray(a, dtype=np.float64)
    return 0.5 * a * (1.0 + erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    """d gelu / d a = Phi(a) + a phi(a)."""
    a = np.asarray(a, dtype=np.float64)
    cdf = 0.5 * (1.0 + erf(a / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)
    return cdf + a * pdf


def init_params(L: int, H1: int, H2: int, seed: int) -> dict:
    """He-uniform weights from the MLP_INIT Philox stream, zero biases (float32 values)."""
    def layer(idx, rows, cols):
        r = np.arange(rows, dtype=np.uint64)[:, None]
        c = np.arange(cols, dtype=np.uint64)[None, :]
        w0, _, _, _ = philox4x32_10(idx, r, c, TAG_MLP_INIT, seed)
        u = ((w0 >> np.uint32(8)).astype(np.float64) + 0.5) * 2.0 ** -24
        bound = math.sqrt(6.0 / cols)
        return (bound * (2.0 * u - 1.0)).astype(np.float32)
    return dict(W1=layer(1, H1, L), b1=np.zeros(H1, np.float32),
                W2=layer(2, H2, H1), b2=np.zeros(H2, np.float32),
                w3=layer(3, 1, H2)[0], b3=np.zeros(1, np.float32))


def forward(params: dict, X) -> dict:
    """X: B x L -> dict(y, a1, h1, a2, h2), float64."""
    X = np.asarray(X, dtype=np.float64)
    p = {k: np.asarray(v, dtype=np.float64) for k, v in params.items()}
    a1 = X @ p["W1"].T + p["b1"]
    h1 = gelu(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(a2)
    y = h2 @ p["w3"] + p["b3"][0]
    return dict(y=y, a1=a1, h1=h1, a2=a2, h2=h2)


def loss_and_grads(params: dict, X, target) -> tuple:
    """Mean squared error over the batch and its gradient for every parameter."""
    X = np.asarray(X, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    p = {k: np.asarray(v, dtype=np.float64) for k, v in params.items()}
    f = forward(params, X)
    B = X.shape[0]
    r = f["y"] - target
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {}
    g["w3"] = f["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    da2 = np.outer(dy, p["w3"]) * gelu_grad(f["a2"])
    g["W2"] = da2.T @ f["h1"]
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * gelu_grad(f["a1"])
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return loss, g


def adam_step(params: dict, grads: dict, m: dict, v: dict, t: int, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> tuple:
    """One Adam update (step number t >= 1).  Returns (params, m, v) as new float64 dicts."""
    newp, newm, newv = {}, {}, {}
    for k in params:
        g = np.asarray(grads[k], dtype=np.float64)
        newm[k] = beta1 * np.asarray(m[k], dtype=np.float64) + (1.0 - beta1) * g
        newv[k] = beta2 * np.asarray(v[k], dtype=np.float64) + (1.0 - beta2) * g * g
        mhat = newm[k] / (1.0 - beta1 ** t)
        vhat = newv[k] / (1.0 - beta2 ** t)
        newp[k] = np.asarray(params[k], dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return newp, newm, newv


def standardise(values) -> tuple:
    """(mean, std) used to standardise the log-MSE targets (population std; 1 if it is 0)."""
    v = np.asarray(values, dtype=np.float64)
    mu = float(v.mean())
    sd = float(v.std())
    return mu, (sd if sd > 0.0 else 1.0)


def recent_rows(batch: int, recent: float) -> int:
    """Rows of a minibatch drawn from the latest append: floor(recent * batch + 1/2)."""
    return int(math.floor(recent * batch + 0.5))


def minibatch_slots(step: int, batch: int, count: int, seed: int, n_recent: int = 0,
                    head: int = 0, last: int = 0, cap: int = 0) -> np.ndarray:
    """Buffer slots of the minibatch of training step `step` (drawn with replacement).

    Row i uses w = word 0 of block (step, i, 0, MINIBATCH).  The first
    batch - n_recent rows are uniform over the count stored pairs, slot
    floor(w count / 2^32); the last n_recent rows are uniform over the `last`
    pairs of the latest append, which end just before slot `head` of the ring
    of capacity `cap`: slot (head - 1 - floor(w last / 2^32)) mod cap.
    """
    i = np.arange(batch, dtype=np.uint64)
    w0, _, _, _ = philox4x32_10(step, i, 0, TAG_MINIBATCH, seed)
    w = w0.astype(np.uint64)
    slots = ((w * np.uint64(count)) >> np.uint64(32)).astype(np.int64)
    if n_recent > 0:
        back = ((w * np.uint64(last)) >> np.uint64(32)).astype(np.int64)
        rec = (head - 1 - back) % cap
        slots[batch - n_recent:] = rec[batch - n_recent:]
    return slots
