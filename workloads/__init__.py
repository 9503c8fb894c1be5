"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module builds INPUT matrices only; it holds none of the principal-minor
arithmetic.  Both the HIP library and the CPU oracle consume what it returns.

Workloads (Sec. V of Simkovic & Ferrero, arXiv:2104.07638: the matrices of a
diagrammatic Monte Carlo step are free propagators between vertices,
M_ij = G0(X_i - X_j) with X = (r, tau)):

* ``lattice_batch``   -- 2D square-lattice tight-binding G0 in imaginary time,
                         vertices uniform on sites and tau in [0, beta);
                         diagonal at tau = 0^- (equal-time density).
* ``keldysh_batch``   -- single-level real-time contour propagators
                         (Sec. V.C): entries G^{a_i a_j}(t_i, t_j) with
                         random times and random Keldysh branch per vertex.
* ``gauss_batch``     -- i.i.d. N(0,1)/sqrt(n) entries (bosonic PPM workload).
* ``inject_stress``   -- near-singular / zero-pivot injections.

All randomness is numpy PCG64 seeded per call; the base seed is 20210415.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BASE_SEED = 20210415


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------------------
# 2D square-lattice free propagator G0(r, tau)
# --------------------------------------------------------------------------------------
@dataclass(frozen=True)
class Lattice:
    L: int = 16
    t: float = 1.0
    mu: float = 0.0
    beta: float = 4.0


def _expit(x):
    # 1 / (1 + exp(-x)) without overflow
    out = np.empty_like(x)
    pos = x >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-x[pos]))
    ex = np.exp(x[~pos])
    out[~pos] = ex / (1.0 + ex)
    return out


def g0_lattice(dx, dy, tau, lat: Lattice) -> np.ndarray:
    """Free lattice propagator by the direct momentum sum (fp64).

    G0(r, tau) = -(1/L^2) sum_k cos(k.r) e^{-xi_k tau} (1 - nF(xi_k))   for 0 < tau < beta
    G0(r, tau) = +(1/L^2) sum_k cos(k.r) e^{-xi_k tau} nF(xi_k)         for -beta < tau <= 0
    with xi_k = -2t(cos kx + cos ky) - mu and nF the Fermi function at 1/beta.
    tau = 0 is taken as 0^- (equal-time density).  The exponential factorises over
    kx and ky, so each entry costs one L x L contraction.
    """
    dx = np.asarray(dx, dtype=np.int64)
    dy = np.asarray(dy, dtype=np.int64)
    tau = np.asarray(tau, dtype=np.float64)
    shape = np.broadcast(dx, dy, tau).shape
    dx, dy, tau = (np.broadcast_to(v, shape).ravel() for v in (dx, dy, tau))
    L = lat.L
    k = 2.0 * np.pi * np.arange(L) / L
    ck = np.cos(k)
    xi = -2.0 * lat.t * (ck[:, None] + ck[None, :]) - lat.mu          # [kx, ky]
    w_pos = -_expit(lat.beta * xi) / (L * L)                          # -(1 - nF)
    w_neg = _expit(-lat.beta * xi) / (L * L)                          # +nF
    out = np.empty(dx.shape[0], dtype=np.float64)
    chunk = 1 << 15
    for s in range(0, dx.shape[0], chunk):
        sl = slice(s, s + chunk)
        ta = tau[sl]
        # e^{-xi tau} = e^{mu tau} e^{2 t tau cos kx} e^{2 t tau cos ky}
        E = np.exp(2.0 * lat.t * ta[:, None] * ck[None, :])            # [e, k]
        Cx = np.cos(np.outer(dx[sl] % L, k))                           # [e, kx]
        Cy = np.cos(np.outer(dy[sl] % L, k))                           # [e, ky]
        Y = Cy * E                                                     # [e, ky]
        pos = ta > 0.0
        Z = np.where(pos[:, None], Y @ w_pos.T, Y @ w_neg.T)           # [e, kx]
        out[sl] = np.exp(lat.mu * ta) * np.einsum("ek,ek->e", Cx * E, Z)
    return out.reshape(shape)


def lattice_vertices(B, n, lat: Lattice, seed):
    """B configurations of n vertices: site uniform on the L x L torus, tau ~ U[0, beta)."""
    rng = _rng(seed)
    xy = rng.integers(0, lat.L, size=(B, n, 2))
    tau = rng.random((B, n)) * lat.beta
    return xy, tau


def lattice_matrices(xy, tau, lat: Lattice) -> np.ndarray:
    """M_ij = G0(r_i - r_j, tau_i - tau_j) for each configuration (diagonal at tau = 0^-)."""
    xy = np.asarray(xy)
    tau = np.asarray(tau, dtype=np.float64)
    dx = xy[:, :, None, 0] - xy[:, None, :, 0]
    dy = xy[:, :, None, 1] - xy[:, None, :, 1]
    dt = tau[:, :, None] - tau[:, None, :]
    return g0_lattice(dx, dy, dt, lat)


def lattice_batch(B, n, lat: Lattice = Lattice(), seed=BASE_SEED) -> np.ndarray:
    """(B, n, n) fp64 propagator matrices for B random vertex configurations."""
    xy, tau = lattice_vertices(B, n, lat, seed)
    return lattice_matrices(xy, tau, lat)


def lattice_ragged(B, n_lo, n_hi, lat: Lattice = Lattice(), seed=BASE_SEED):
    """B matrices with orders uniform in {n_lo..n_hi}; returns (list of matrices, orders)."""
    rng = _rng(seed + 7919)
    ns = rng.integers(n_lo, n_hi + 1, size=B)
    mats = []
    for nn in range(n_lo, n_hi + 1):
        idx = np.nonzero(ns == nn)[0]
        if idx.size == 0:
            continue
        Ms = lattice_batch(idx.size, nn, lat, seed=seed + 1000 * nn)
        mats.extend(zip(idx.tolist(), Ms))
    mats.sort(key=lambda p: p[0])
    return [m for _, m in mats], ns.astype(np.int32)


# --------------------------------------------------------------------------------------
# Real-time (Keldysh) single-level propagators, Sec. V.C
# --------------------------------------------------------------------------------------
def keldysh_batch(B, n, eps=0.5, n0=0.3, tmax=10.0, seed=BASE_SEED) -> np.ndarray:
    """(B, n, n) complex128 contour-ordered propagators of one level.

    G^>(t,t') = -i (1 - n0) e^{-i eps (t - t')},  G^<(t,t') = +i n0 e^{-i eps (t - t')}.
    Branch + is time ordered, branch - anti-time ordered; G^{+-} = G^<, G^{-+} = G^>.
    Equal times (and the diagonal) use G^<.
    """
    rng = _rng(seed)
    t = rng.random((B, n)) * tmax
    br = rng.integers(0, 2, size=(B, n))            # 0 -> '+', 1 -> '-'
    dt = t[:, :, None] - t[:, None, :]
    ph = np.exp(-1j * eps * dt)
    g_gt = -1j * (1.0 - n0) * ph
    g_lt = 1j * n0 * ph
    ai = br[:, :, None]
    aj = br[:, None, :]
    later = dt > 0.0                                  # t_i later than t_j
    earlier = dt < 0.0
    M = np.where((ai == 0) & (aj == 0), np.where(later, g_gt, g_lt), 0.0)
    M = M + np.where((ai == 1) & (aj == 1), np.where(earlier, g_gt, g_lt), 0.0)
    M = M + np.where((ai == 0) & (aj == 1), g_lt, 0.0)
    M = M + np.where((ai == 1) & (aj == 0), g_gt, 0.0)
    return np.ascontiguousarray(M.astype(np.complex128))


def keldysh_block(B, n, eps=0.5, n0=0.3, tmax=10.0, seed=BASE_SEED) -> np.ndarray:
    """(B, 2n, 2n) complex128 Keldysh block matrices (Sec. V.C, real-time DiagMC).

    Block (i, j) is [[G^{++}, G^{+-}], [G^{-+}, G^{--}]] at t_i - t_j with the propagators
    of ``keldysh_batch``: row/column 2i + a is vertex i on branch a (0 = '+', 1 = '-').
    Keeping one row of every block (row 2i + alpha_i) gives that function's matrix for the
    branch assignment alpha.  Times t_i ~ U[0, tmax).
    """
    rng = _rng(seed)
    t = rng.random((B, n)) * tmax
    dt = t[:, :, None] - t[:, None, :]
    ph = np.exp(-1j * eps * dt)
    g_gt = -1j * (1.0 - n0) * ph
    g_lt = 1j * n0 * ph
    later = dt > 0.0
    earlier = dt < 0.0
    out = np.empty((B, 2 * n, 2 * n), dtype=np.complex128)
    out[:, 0::2, 0::2] = np.where(later, g_gt, g_lt)      # ++ : time ordered
    out[:, 1::2, 1::2] = np.where(earlier, g_gt, g_lt)    # -- : anti-time ordered
    out[:, 0::2, 1::2] = g_lt                              # +- = G^<
    out[:, 1::2, 0::2] = g_gt                              # -+ = G^>
    return out


def keldysh_config(B, n, eps=0.5, n0=0.3, tmax=10.0, seed=BASE_SEED):
    """Return (times, branches) used by ``keldysh_batch`` with the same seed."""
    rng = _rng(seed)
    t = rng.random((B, n)) * tmax
    br = rng.integers(0, 2, size=(B, n))
    return t, br


# --------------------------------------------------------------------------------------
# Gaussian matrices (bosonic permanent workload) and generic helpers
# --------------------------------------------------------------------------------------
def gauss_batch(B, n, seed=BASE_SEED, complex_=False) -> np.ndarray:
    rng = _rng(seed)
    A = rng.standard_normal((B, n, n)) / np.sqrt(n)
    if complex_:
        A = A + 1j * rng.standard_normal((B, n, n)) / np.sqrt(n)
    return np.ascontiguousarray(A)


# --------------------------------------------------------------------------------------
# Stress injections (near-singular pivots, zero diagonal)
# --------------------------------------------------------------------------------------
def inject_stress(A, every=64, seed=BASE_SEED, scale=1e-12):
    """Make every ``every``-th matrix (b = 0, every, 2*every, ...) near-singular.

    Injections alternate between
      (i)  diagonal entry A_kk multiplied by ``scale`` (k = (b // every) mod n);
      (ii) A_ll shifted so that det A[r + {l}] = scale * s * det A[r] for a random
           nonempty r not containing l (s = max |A_ij|): the 1 x 1 Schur complement
           of A[r + {l}] over A[r] becomes tiny, whatever pivot order is used.
    The shift in (ii) needs det A[r + {l}] / det A[r] = A_ll - A[l,r] A[r]^{-1} A[r,l],
    which is computed here with numpy's solver (input construction, not the method).
    Returns (A_new, list of (b, kind, detail)).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    B, n, _ = A.shape
    rng = _rng(seed + 104729)
    log = []
    for j, b in enumerate(range(0, B, every)):
        s = np.abs(A[b]).max()
        if j % 2 == 0 or n < 2:
            k = (b // every) % n
            A[b, k, k] *= scale
            log.append((b, "diag", k))
        else:
            l = int(rng.integers(0, n))
            others = [i for i in range(n) if i != l]
            size = int(rng.integers(1, n))
            r = sorted(rng.choice(others, size=size, replace=False).tolist())
            Arr = A[b][np.ix_(r, r)]
            ratio = A[b, l, l] - A[b, l, r] @ np.linalg.solve(Arr, A[b, r, l])
            A[b, l, l] += scale * s - ratio
            log.append((b, "pivot", (l, tuple(r))))
    return A, log


def zero_diagonal(A):
    A = np.array(A, copy=True)
    idx = np.arange(A.shape[-1])
    A[..., idx, idx] = 0.0
    return A


# --------------------------------------------------------------------------------------
# Monte Carlo over vertex configurations with a learned proposal (inputs only)
# --------------------------------------------------------------------------------------
@dataclass(frozen=True)
class McModel:
    """Vertex configurations of the imaginary-time lattice expansion.

    A configuration is n vertices; vertex i sits on lattice site s_i = y_i L + x_i and
    at imaginary time tau_i = (j_i + 1/2) beta / n_tau on a grid of n_tau points.  A
    vertex is packed as ``s | (j << 16)``.  The learned proposal groups the n_tau time
    points into n_bin equal bins and mixes in a fraction ``eps`` of the uniform proposal.
    ``resolve`` > 0 gives weight zero to configurations whose connected sum is below
    resolve times the rounding scale of the recursion.
    """
    n: int = 10
    L: int = 16
    t: float = 1.0
    mu: float = 0.0
    beta: float = 4.0
    n_tau: int = 128
    n_bin: int = 16
    eps: float = 0.1
    resolve: float = 0.0

    @property
    def lattice(self) -> Lattice:
        return Lattice(L=self.L, t=self.t, mu=self.mu, beta=self.beta)

    @property
    def d_in(self) -> int:
        return 3 * (self.n - 1)

    @property
    def d_out(self) -> int:
        return self.L * self.L + self.n_bin


def mc_g0_table(m: McModel) -> np.ndarray:
    """G0 on the vertex grid: row d + n_tau - 1 holds tau difference d beta / n_tau
    (d in [-(n_tau-1), n_tau-1]; d = 0 is 0^-), column dy*L + dx holds the site
    difference (dx, dy) taken mod L.  Shape (2 n_tau - 1, L^2), fp64."""
    d = np.arange(-(m.n_tau - 1), m.n_tau)
    s = np.arange(m.L * m.L)
    tau = d[:, None] * (m.beta / m.n_tau)
    return np.ascontiguousarray(g0_lattice((s % m.L)[None, :], (s // m.L)[None, :], tau, m.lattice))


def pack_vertex(site, tidx):
    return (np.asarray(site, dtype=np.uint32) | (np.asarray(tidx, dtype=np.uint32) << np.uint32(16)))


def mc_initial_states(W, m: McModel, seed=BASE_SEED) -> np.ndarray:
    """W configurations of n vertices, sites and time points uniform; uint32 (W, n)."""
    rng = _rng(seed + 31337)
    site = rng.integers(0, m.L * m.L, size=(W, m.n))
    tidx = rng.integers(0, m.n_tau, size=(W, m.n))
    return np.ascontiguousarray(pack_vertex(site, tidx))


def mc_cluster_states(W, m: McModel, seed=BASE_SEED, width: int = 2, t_width: int = 8) -> np.ndarray:
    """W configurations whose n vertices sit in a width x width block of sites and
    t_width consecutive time points around a random corner (the compact region where
    |c[V]| is large and resolved in fp64; uniformly spread vertices give |c[V]| at the
    rounding level of the recursion's terms).  uint32 (W, n)."""
    rng = _rng(seed + 4242)
    x0 = rng.integers(0, m.L, size=(W, 1))
    y0 = rng.integers(0, m.L, size=(W, 1))
    tw = min(t_width, m.n_tau)
    t0 = rng.integers(0, m.n_tau - tw + 1, size=(W, 1))
    x = (x0 + rng.integers(0, width, size=(W, m.n))) % m.L
    y = (y0 + rng.integers(0, width, size=(W, m.n))) % m.L
    t = t0 + rng.integers(0, tw, size=(W, m.n))
    return np.ascontiguousarray(pack_vertex(y * m.L + x, t))


MLP_HIDDEN = 128


def mlp_dims(d_in: int, d_out: int):
    """Padded sizes of the proposal network: inputs to a multiple of 16 (at least 16),
    outputs to a multiple of 16."""
    dp = max(16, -(-d_in // 16) * 16)
    op = -(-d_out // 16) * 16
    return dp, op


def mlp_param_count(d_in: int, d_out: int) -> int:
    """fp32 parameters in the packed order W1 (H x Dp) | W2 (H x H) | W3 (Op x H) |
    b1 (H) | b2 (H) | b3 (Op), matrices row-major [out][in]."""
    dp, op = mlp_dims(d_in, d_out)
    H = MLP_HIDDEN
    return H * dp + H * H + op * H + H + H + op


def mlp_init(d_in: int, d_out: int, seed=BASE_SEED, gain: float = 1.0) -> np.ndarray:
    """Packed fp32 parameters: Glorot-uniform weights on the logical block (scaled by
    ``gain``), zero padding rows/columns and zero biases."""
    rng = _rng(seed + 271828)
    dp, op = mlp_dims(d_in, d_out)
    H = MLP_HIDDEN
    p = np.zeros(mlp_param_count(d_in, d_out), dtype=np.float32)
    off = 0
    # (stored rows, stored cols, logical rows, logical cols)
    for rows, cols, lr, lc in ((H, dp, H, d_in), (H, H, H, H), (op, H, d_out, H)):
        lim = gain * np.sqrt(6.0 / (lr + lc))
        w = np.zeros((rows, cols), dtype=np.float32)
        w[:lr, :lc] = rng.uniform(-lim, lim, size=(lr, lc))
        p[off:off + rows * cols] = w.ravel()
        off += rows * cols
    return p
