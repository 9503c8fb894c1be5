"""Proposal network -- oracle side, TEST INFRASTRUCTURE ONLY.

Plain fp64 numpy forward and backward passes of the two-hidden-layer tanh network that
drives the learned Monte Carlo proposal, and the Adam update (Kingma & Ba, ICLR 2015,
Algorithm 1, with bias correction).  The network as the library defines it:

    x_b  = bf16(x)                              input features, rounded to bfloat16
    h1   = tanh(bf16(W1) x_b + b1)              hidden width H = 128
    h2   = tanh(bf16(W2) bf16(h1) + b2)
    out  = bf16(W3) bf16(h2) + b3

Weights are rounded to bfloat16, biases stay fp32, hidden activations are rounded to
bfloat16 where they enter the next product.  ``rounding=False`` evaluates the same
network without any rounding (used to pin the gradients against finite differences).
The gradient is the derivative of ``out`` with the rounding steps taken as the identity
(the tanh derivative uses the unrounded activation).

Parameters are one packed fp32 vector, matrices row-major [out][in]:
W1 (H x Dp) | W2 (H x H) | W3 (Op x H) | b1 (H) | b2 (H) | b3 (Op), with Dp and Op the
input and output sizes padded to multiples of 16 (Dp >= 16).
"""
from __future__ import annotations

import numpy as np

HIDDEN = 128


def dims(d_in: int, d_out: int):
    dp = max(16, -(-d_in // 16) * 16)
    op = -(-d_out // 16) * 16
    return dp, op


def unpack(p, d_in: int, d_out: int):
    """Views (W1, W2, W3, b1, b2, b3) into the packed parameter vector."""
    dp, op = dims(d_in, d_out)
    H = HIDDEN
    sizes = [(H, dp), (H, H), (op, H), (H,), (H,), (op,)]
    out, off = [], 0
    for s in sizes:
        cnt = int(np.prod(s))
        out.append(p[off:off + cnt].reshape(s))
        off += cnt
    if off != p.shape[0]:
        raise ValueError("parameter vector has the wrong length")
    return out


def bf16(x):
    """Round to bfloat16 (round to nearest, ties to even) via fp32; returned as fp64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, x, d_in: int, d_out: int, rounding: bool = True):
    """x: (B, Dp) features -> (out (B, Op), cache)."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3, b1, b2, b3 = unpack(np.asarray(p, dtype=np.float64), d_in, d_out)
    W1, W2, W3 = r(W1), r(W2), r(W3)
    xb = r(x)
    h1 = np.tanh(xb @ W1.T + b1)
    h1b = r(h1)
    h2 = np.tanh(h1b @ W2.T + b2)
    h2b = r(h2)
    out = h2b @ W3.T + b3
    cache = dict(x=xb, h1=h1, h1b=h1b, h2=h2, h2b=h2b, W1=W1, W2=W2, W3=W3, d_in=d_in, d_out=d_out)
    return out, cache


def backward(cache, dout):
    """Gradient of sum(out * dout) with respect to the packed parameters (fp64)."""
    dout = np.asarray(dout, dtype=np.float64)
    gW3 = dout.T @ cache["h2b"]
    gb3 = dout.sum(0)
    dz2 = (dout @ cache["W3"]) * (1.0 - cache["h2"] ** 2)
    gW2 = dz2.T @ cache["h1b"]
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ cache["W2"]) * (1.0 - cache["h1"] ** 2)
    gW1 = dz1.T @ cache["x"]
    gb1 = dz1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gW2, gW3, gb1, gb2, gb3)])


def adam(p, m, v, g, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step number t >= 1; returns (p, m, v) as new fp64 arrays."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return np.asarray(p, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
