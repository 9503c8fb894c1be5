"""Monte Carlo over vertex configurations -- oracle side, TEST INFRASTRUCTURE ONLY.

Target distribution: pi(X) proportional to |c[V](X)|, the connected sum over the full
vertex set V of a configuration X (Sec. V.A, Eq. (recursion)) with the CDet weights
a[S] = det(M[S])^2 (both spins share M) and M_ij = G0(X_i - X_j) (Sec. V.A), taken from
the tabulated propagator of ``workloads.mc_g0_table``.  With model.resolve > 0 the weight
is zero where |c[V]| < resolve * d[V], d[V] = |a[V]| + sum_T |c[T]| |a[V - T]| the
recursion's rounding scale (``oracle.cs_scale``): there c[V] is not resolved in fp64.

One step per walker (the paper defines the weight, not the sampler; this is the
project's design):
  1. choose the moved vertex k uniformly;
  2. the context is the other n-1 vertices sorted by (time point, site); its features
     are (x/L, y/L, (j+1/2)/n_tau) per context vertex, rounded to bfloat16;
  3. propose v' either uniformly over sites x time points, or from the network:
     with probability eps uniformly, otherwise site ~ softmax(site logits),
     bin ~ softmax(bin logits), time point uniform inside the bin;
     q~(v|ctx) = (1-eps) p_site(s) p_bin(b) / (n_tau/n_bin) + eps / (L^2 n_tau);
  4. accept with probability min(1, |c(X')| q~(v_k|ctx) / (|c(X)| q~(v'|ctx))): exact,
     because the context is the same in both directions.
Random numbers: Philox4x64-10 (``oracle.philox``), key (seed, 0), counter
(walker, step, call, 0).  Call 0: k, eps test, uniform site, uniform time point.
Call 1: site draw, bin draw, time point inside the bin, acceptance.
Categorical draws take the first index whose running sum exceeds u * total.
"""
from __future__ import annotations

import numpy as np

from . import connected_sums, cs_scale, minors
from . import mlp as _mlp
from . import philox


def unpack(v):
    v = np.asarray(v, dtype=np.uint32)
    return (v & np.uint32(0xFFFF)).astype(np.int64), (v >> np.uint32(16)).astype(np.int64)


def pack(site, tidx):
    return (np.asarray(site, dtype=np.uint32) | (np.asarray(tidx, dtype=np.uint32) << np.uint32(16)))


def matrices(model, g0, states):
    """(W, n, n) propagator matrices of the configurations ``states`` (W, n)."""
    site, t = unpack(states)
    L = model.L
    x, y = site % L, site // L
    dx = (x[:, :, None] - x[:, None, :]) % L
    dy = (y[:, :, None] - y[:, None, :]) % L
    d = t[:, :, None] - t[:, None, :] + model.n_tau - 1
    return np.ascontiguousarray(np.asarray(g0)[d, dy * L + dx])


def full_connected_sum(model, g0, states):
    """c[V] for each configuration: minors -> a = det^2 -> rooted recursion."""
    m = minors(matrices(model, g0, states))
    c = connected_sums(m * m, mode=0)
    return c[:, -1]


def weight(model, g0, states):
    """(log of the weight, sign) per configuration: log|c[V]| and sign(c[V]), or
    (-inf, 0) for a zero, non-finite or unresolved c[V]."""
    m = minors(matrices(model, g0, states))
    a = m * m
    c = connected_sums(a, mode=0)
    cv = c[:, -1]
    ok = np.isfinite(cv) & (cv != 0.0)
    if model.resolve > 0.0:
        d = cs_scale(a, c, mode=0)[:, -1]
        ok &= np.abs(cv) >= model.resolve * d
    lw = np.full(cv.shape, -np.inf)
    lw[ok] = np.log(np.abs(cv[ok]))
    return lw, np.where(ok, np.sign(cv), 0.0).astype(np.int8)


def log_abs(c):
    c = np.asarray(c, dtype=np.float64)
    out = np.full(c.shape, -np.inf)
    ok = np.isfinite(c) & (c != 0.0)
    out[ok] = np.log(np.abs(c[ok]))
    return out


def draws(seed, W, step):
    w = np.arange(W)
    return philox.mc_draws(seed, w, step, 0), philox.mc_draws(seed, w, step, 1)


def moved_vertex(model, d0):
    return philox.below(d0[:, 0], model.n)


def context(model, states, k):
    """Other n-1 vertices sorted by (time point, site) = by the packed value."""
    W, n = states.shape
    keep = np.ones((W, n), dtype=bool)
    keep[np.arange(W), k] = False
    ctx = states[keep].reshape(W, n - 1)
    return np.sort(ctx, axis=1)


def features(model, ctx):
    """bfloat16-rounded (x/L, y/L, (j+1/2)/n_tau) per context vertex, zero padded."""
    W = ctx.shape[0]
    dp, _ = _mlp.dims(model.d_in, model.d_out)
    site, t = unpack(ctx)
    f = np.zeros((W, dp))
    f[:, 0:3 * ctx.shape[1]:3] = (site % model.L) / model.L
    f[:, 1:3 * ctx.shape[1]:3] = (site // model.L) / model.L
    f[:, 2:3 * ctx.shape[1]:3] = (t + 0.5) / model.n_tau
    return _mlp.bf16(f)


def categorical(p, u):
    """Row-wise first index whose running sum exceeds u * total (else the last positive
    entry of the row).  p: (W, m) nonnegative, u: (W,)."""
    cs = np.cumsum(p, axis=1)
    j = (cs <= (u * cs[:, -1])[:, None]).sum(axis=1)
    last = p.shape[1] - 1 - np.argmax(p[:, ::-1] > 0, axis=1)
    return np.where(j >= p.shape[1], last, j)


def _softmax_parts(model, logits):
    L2 = model.L * model.L
    lg = np.asarray(logits, dtype=np.float64)
    s = lg[:, :L2]
    b = lg[:, L2:L2 + model.n_bin]
    ps = np.exp(s - s.max(axis=1, keepdims=True))
    pb = np.exp(b - b.max(axis=1, keepdims=True))
    return ps, pb


def log_q(model, logits, site, tidx):
    """log q~(v | ctx) of the mixed learned proposal, one vertex per context row."""
    ps, pb = _softmax_parts(model, logits)
    r = np.arange(ps.shape[0])
    per_bin = model.n_tau // model.n_bin
    q = ((1.0 - model.eps) * ps[r, site] / ps.sum(axis=1) * pb[r, tidx // per_bin] / pb.sum(axis=1) / per_bin
         + model.eps / (model.L * model.L * model.n_tau))
    return np.log(q)


def propose(model, states, k, d0, d1, logits=None):
    """Proposed vertex (packed) and log q~(v_k) - log q~(v') per walker."""
    W = states.shape[0]
    L2 = model.L * model.L
    us = philox.below(d0[:, 2], L2)
    ut = philox.below(d0[:, 3], model.n_tau)
    if logits is None:
        return pack(us, ut), np.zeros(W)
    per_bin = model.n_tau // model.n_bin
    ps, pb = _softmax_parts(model, logits)
    ls = categorical(ps, philox.uniform(d1[:, 0]))
    lb = categorical(pb, philox.uniform(d1[:, 1]))
    lt = lb * per_bin + philox.below(d1[:, 2], per_bin)
    uni = philox.uniform(d0[:, 1]) < model.eps
    s = np.where(uni, us, ls)
    t = np.where(uni, ut, lt)
    cur_site, cur_t = unpack(states[np.arange(W), k])
    logq = log_q(model, logits, cur_site, cur_t) - log_q(model, logits, s, t)
    return pack(s, t), logq


def accept(logw, logc_prop, logq, u):
    """Metropolis-Hastings decision in log space: accept iff log u < log R, with
    log R = log|c'| - log|c| + logq; a zero proposal weight is never accepted and a
    zero current weight always yields to a nonzero proposal."""
    logw = np.asarray(logw, dtype=np.float64)
    logc_prop = np.asarray(logc_prop, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        logR = logc_prop - logw + logq
        acc = np.isfinite(logc_prop) & (np.isneginf(logw) | (np.log(u) < logR))
    return acc


def accept_probability(logw, logc_prop, logq):
    """P(accept) of ``accept`` for a uniform u: min(1, exp(log R))."""
    if not np.isfinite(logc_prop):
        return 0.0
    if np.isneginf(logw):
        return 1.0
    return float(min(1.0, np.exp(logc_prop - logw + logq)))


def step(model, g0, states, logw, sign, seed, step_no, params=None, logits=None):
    """One step for every walker.  ``params`` (packed network) gives the learned
    proposal; ``logits`` overrides the network output (fp32 values); neither: uniform."""
    states = np.array(states, dtype=np.uint32, copy=True)
    W = states.shape[0]
    d0, d1 = draws(seed, W, step_no)
    k = moved_vertex(model, d0)
    ctx = context(model, states, k)
    feat = features(model, ctx)
    if logits is None and params is not None:
        logits, _ = _mlp.forward(params, feat, model.d_in, model.d_out)
    prop, logq = propose(model, states, k, d0, d1, logits)
    new = states.copy()
    new[np.arange(W), k] = prop
    lc, sg = weight(model, g0, new)
    acc = accept(logw, lc, logq, philox.uniform(d1[:, 3]))
    out_states = np.where(acc[:, None], new, states)
    out_logw = np.where(acc, lc, logw)
    out_sign = np.where(acc, sg, sign).astype(np.int8)
    return dict(k=k, feat=feat, logits=logits, prop=prop, logq=logq, logc_prop=lc,
                accept=acc, states=out_states, logw=out_logw, sign=out_sign)


def loss_grad(model, logits, prop, logc_prop, clip: float = 30.0):
    """Regression of site logit + bin logit on log|c'| (clipped below at max - clip):
    returns (loss, dout) for the mean squared error over the W walkers."""
    logits = np.asarray(logits, dtype=np.float64)
    W = logits.shape[0]
    L2 = model.L * model.L
    site, t = unpack(prop)
    b = t // (model.n_tau // model.n_bin)
    y = np.asarray(logc_prop, dtype=np.float64)
    dout = np.zeros_like(logits)
    fin = np.isfinite(y)
    if not fin.any():
        return 0.0, dout
    floor = y[fin].max() - clip
    y = np.where(fin, np.maximum(y, floor), floor)
    r = np.arange(W)
    pred = logits[r, site] + logits[r, L2 + b]
    g = 2.0 * (pred - y) / W
    dout[r, site] += g
    dout[r, L2 + b] += g
    return float(np.mean((pred - y) ** 2)), dout


def enumerate_states(model):
    """All (L^2 n_tau)^n labelled configurations (tiny models only), packed (S, n)."""
    V = model.L * model.L * model.n_tau
    S = V ** model.n
    if S > 1 << 16:
        raise ValueError("state space too large to enumerate")
    idx = np.arange(S)
    vi = np.stack([(idx // V ** i) % V for i in range(model.n)], axis=1)
    L2 = model.L * model.L
    return pack(vi % L2, vi // L2)
