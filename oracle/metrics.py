"""Error metrics (test and benchmark infrastructure) for comparing principal minors with the oracle.

Plain relative error is undefined for (near-)zero minors, so the parity gate is the
mixed metric  e_S = |x_S - ref_S| / max(|ref_S|, H_S)  with the Hadamard bound
H_S = prod_{i in S} ||A[i, S]||_2 >= |det A[S]|  (e_S = 0 when x_S == ref_S)."""
import numpy as np


def _row_scaled_squares(A):
    """|A_ij|^2 / m_i^2 and log m_i with m_i = max_j |A_ij| (1 for a zero row), so that the
    squares neither overflow nor underflow for any finite entries."""
    mag = np.abs(A)
    m = mag.max(axis=-1, keepdims=True)
    m = np.where(m > 0, m, 1.0)
    return (mag / m) ** 2, np.log(m[..., 0])


def hadamard_bounds(A):
    """H[m] = prod_{i in S_m} ||A[i, S_m]||_2 for every mask m, for one (n, n) matrix."""
    A = np.asarray(A)
    n = A.shape[0]
    sq, logm = _row_scaled_squares(A)
    nm = 1 << n
    logH = np.zeros(nm)
    masks = np.arange(nm)
    for i in range(n):
        rows = np.zeros(1)
        for j in range(n):
            rows = np.concatenate([rows, rows + sq[i, j]])
        with np.errstate(divide="ignore"):
            lr = 0.5 * np.log(rows) + logm[i]
        inS = (masks >> i) & 1
        logH = logH + np.where(inS == 1, lr, 0.0)
    return np.exp(logH)


def _norm2(x):
    """||x||_2 computed as m ||x / m||_2, m = max |x_j|, free of overflow and underflow."""
    m = np.max(np.abs(x)) if x.size else 0.0
    return 0.0 if m == 0 else m * np.sqrt(np.sum((np.abs(x) / m) ** 2))


def hadamard_at(A, masks):
    """H_S for the listed masks only, by explicit products of row norms (log-summed)."""
    A = np.asarray(A)
    n = A.shape[0]
    out = np.empty(len(masks))
    for t, m in enumerate(masks):
        r = [k for k in range(n) if m >> k & 1]
        with np.errstate(divide="ignore"):
            out[t] = np.exp(np.sum([np.log(_norm2(A[i, r])) for i in r])) if r else 1.0
    return out


def mixed_err(x, ref, H):
    x = np.asarray(x)
    ref = np.asarray(ref)
    diff = np.abs(x - ref)
    den = np.maximum(np.abs(ref), H)
    with np.errstate(invalid="ignore", divide="ignore"):
        e = np.where(diff == 0, 0.0, diff / np.where(den == 0, np.finfo(float).tiny, den))
    e = np.where(np.isfinite(x) | ~np.isfinite(ref), e, np.inf)
    return e


def max_mixed_err(X, REF, A):
    """max over a batch of the mixed metric; X, REF are (B, 2^n), A is (B, n, n)."""
    worst = 0.0
    for b in range(X.shape[0]):
        e = mixed_err(X[b], REF[b], hadamard_bounds(A[b]))
        worst = max(worst, float(np.max(e)))
    return worst


def hadamard_bounds_batch(A):
    """hadamard_bounds for a (B, n, n) batch."""
    A = np.asarray(A)
    B, n, _ = A.shape
    sq, logm = _row_scaled_squares(A)
    nm = 1 << n
    masks = np.arange(nm)
    logH = np.zeros((B, nm))
    for i in range(n):
        rows = np.zeros((B, 1))
        for j in range(n):
            rows = np.concatenate([rows, rows + sq[:, i, j:j + 1]], axis=1)
        with np.errstate(divide="ignore"):
            lr = 0.5 * np.log(rows) + logm[:, i:i + 1]
        logH = logH + np.where(((masks >> i) & 1) == 1, lr, 0.0)
    return np.exp(logH)


def cdet_tolerance(A, m, c, eps_minor=1e-10, eps_cs=1e-10, mode=0):
    """Tolerance for connected sums computed from independently rounded minors of A:
    each minor may be off by eps_minor * max(|m|, H_S) (the minors' own gate), which
    gives weight errors da = 2|m| dm + dm^2 for a = m^2, propagated through the
    recursion to first order; plus eps_cs times the recursion's own rounding scale."""
    from . import cs_input_bound, cs_scale
    A = np.asarray(A)
    H = hadamard_bounds_batch(A)
    dm = eps_minor * np.maximum(np.abs(m), H)
    a = m * m
    da = 2.0 * np.abs(m) * dm + dm * dm
    return eps_cs * cs_scale(a, c, mode) + cs_input_bound(a, c, da, mode)
