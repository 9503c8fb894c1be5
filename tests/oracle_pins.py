"""Pins for the CPU oracle: facts fixed by the paper or by mathematics, not by the oracle.

Each ``pin_*`` function takes the oracle functions to check (so that the same
battery can run against deliberately broken builds) and raises AssertionError
when the fact does not hold.  None of them re-types the oracle's formulas: they
use closed forms, invariants, brute force over permutations or set partitions,
independent library routines (numpy.linalg.det, numpy.poly) or mpmath at 40
digits.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def submask_rows(m, n):
    return [k for k in range(n) if m >> k & 1]


def perm_sign(p):
    p = list(p)
    s = 1
    seen = [False] * len(p)
    for i in range(len(p)):
        if seen[i]:
            continue
        j, L = i, 0
        while not seen[j]:
            seen[j] = True
            j = p[j]
            L += 1
        if L % 2 == 0:
            s = -s
    return s


def leibniz_det(M):
    k = M.shape[0]
    tot = 0.0
    for p in itertools.permutations(range(k)):
        prod = 1.0
        for i in range(k):
            prod = prod * M[i, p[i]]
        tot = tot + perm_sign(p) * prod
    return tot


def brute_perm(M):
    k = M.shape[0]
    tot = 0.0
    for p in itertools.permutations(range(k)):
        prod = 1.0
        for i in range(k):
            prod *= M[i, p[i]]
        tot += prod
    return tot


def set_partitions(items):
    items = list(items)
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in set_partitions(rest):
        # put `first` in a new block or into an existing block
        yield [[first]] + part
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]


def close(a, b, rtol, atol=0.0):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.all(np.abs(a - b) <= atol + rtol * np.abs(b))


# ----------------------------------------------------------------------------------
# principal minors (Sec. II)
# ----------------------------------------------------------------------------------
def minors_via_masks(oracle_mod, A, lib=None):
    """All principal minors through the mask-list entry point ``minors_at`` (every mask
    listed), for single matrices or batches, so that the same pins check it."""
    A = np.asarray(A, dtype=np.float64)
    single = A.ndim == 2
    Ab = A[None] if single else A
    masks = np.arange(1 << Ab.shape[-1], dtype=np.uint32)
    out = np.stack([oracle_mod.minors_at(a, masks, lib=lib) for a in Ab])
    return out[0] if single else out


def pin_minors_golden_mask(minors):
    """Sec. II bit-mask example: mask 13 <-> rows {1,3,4} (1-based)."""
    g = json.load(open(os.path.join(GOLDEN, "mask_convention.json")))
    A = _rng(11).standard_normal((5, 5))
    out = minors(A)
    rows = g["rows_0based"]
    assert [r + 1 for r in rows] == g["rows_1based"]
    assert submask_rows(g["mask"], 5) == rows
    ref = leibniz_det(A[np.ix_(rows, rows)])
    assert abs(out[g["mask"]] - ref) <= 1e-13 * max(1.0, abs(ref)), (out[g["mask"]], ref)


def pin_minors_empty_and_diag(minors):
    A = _rng(1).standard_normal((6, 6))
    out = minors(A)
    assert out[0] == 1.0
    for k in range(6):
        assert out[1 << k] == A[k, k]


def pin_minors_triangular(minors):
    rng = _rng(2)
    A = np.triu(rng.standard_normal((7, 7))) + 2.0 * np.eye(7)
    for M in (A, A.T.copy()):
        out = minors(M)
        d = np.diag(M)
        ref = np.array([np.prod(d[submask_rows(m, 7)]) for m in range(1 << 7)])
        assert close(out, ref, 1e-13), np.max(np.abs(out - ref))


def pin_minors_leibniz(minors):
    rng = _rng(3)
    for n in (1, 2, 3, 4, 5, 6):
        A = rng.standard_normal((n, n))
        out = minors(A)
        for m in range(1 << n):
            r = submask_rows(m, n)
            ref = leibniz_det(A[np.ix_(r, r)]) if r else 1.0
            assert abs(out[m] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, m, out[m], ref)


def pin_minors_det_I_plus_A(minors):
    """sum_S det A[S] = det(I + A) (expansion of det(I+A) by multilinearity)."""
    rng = _rng(4)
    for n in (3, 8, 11):
        A = rng.standard_normal((n, n)) / np.sqrt(n)
        out = minors(A)
        ref = np.linalg.det(np.eye(n) + A)
        assert abs(out.sum() - ref) <= 1e-10 * max(1.0, np.abs(out).sum()), (n, out.sum(), ref)


def pin_minors_charpoly(minors):
    """Sum of the k x k principal minors = k-th coefficient of det(lambda I + A)."""
    rng = _rng(5)
    n = 9
    A = rng.standard_normal((n, n))
    out = minors(A)
    pc = np.poly(A)            # det(lambda I - A) = sum_k pc[k] lambda^(n-k)
    sizes = np.array([bin(m).count("1") for m in range(1 << n)])
    for k in range(n + 1):
        ek = out[sizes == k].sum()
        ref = (-1) ** k * pc[k]
        assert abs(ek - ref) <= 1e-9 * max(1.0, abs(ref)), (k, ek, ref)


def pin_minors_invariances(minors):
    rng = _rng(6)
    n = 8
    A = rng.standard_normal((n, n))
    out = minors(A)
    d = np.exp(rng.standard_normal(n))
    assert close(minors(A.T.copy()), out, 1e-12, 1e-13)
    assert close(minors((d[:, None] * A) / d[None, :]), out, 1e-11, 1e-13)
    alpha = -1.7
    sizes = np.array([bin(m).count("1") for m in range(1 << n)])
    assert close(minors(alpha * A), out * alpha ** sizes, 1e-12, 1e-13)


def pin_minors_block_diag(minors):
    rng = _rng(7)
    A1 = rng.standard_normal((3, 3))
    A2 = rng.standard_normal((4, 4))
    A = np.zeros((7, 7))
    A[:3, :3] = A1
    A[3:, 3:] = A2
    out = minors(A)
    o1 = minors(A1)
    o2 = minors(A2)
    ref = np.array([o1[m & 7] * o2[m >> 3] for m in range(1 << 7)])
    assert close(out, ref, 1e-12, 1e-14)


def pin_minors_mpmath_near_singular(minors):
    """Near-singular submatrix: compare with 40-digit determinants (mpmath)."""
    import mpmath
    mpmath.mp.dps = 40
    rng = _rng(8)
    n = 7
    A = rng.standard_normal((n, n))
    # make A[{0,2,5}] nearly singular: third row = combination of the first two + 1e-11
    A[5, [0, 2, 5]] = 0.3 * A[0, [0, 2, 5]] - 1.1 * A[2, [0, 2, 5]]
    A[5, 5] += 1e-11
    out = minors(A)
    for m in range(1 << n):
        r = submask_rows(m, n)
        if not r:
            continue
        M = mpmath.matrix([[mpmath.mpf(float(A[i, j])) for j in r] for i in r])
        ref = float(mpmath.det(M))
        scale = float(np.prod([np.linalg.norm(A[i, r]) for i in r]))   # Hadamard bound
        assert abs(out[m] - ref) <= 1e-13 * scale, (m, out[m], ref, scale)


MINOR_PINS = [pin_minors_golden_mask, pin_minors_empty_and_diag, pin_minors_triangular,
              pin_minors_leibniz, pin_minors_det_I_plus_A, pin_minors_charpoly,
              pin_minors_invariances, pin_minors_block_diag, pin_minors_mpmath_near_singular]


# ----------------------------------------------------------------------------------
# complex minors (Sec. V.C)
# ----------------------------------------------------------------------------------
def pin_cminors_leibniz(cminors):
    rng = _rng(21)
    for n in (1, 2, 3, 4, 5):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        out = cminors(A)
        for m in range(1 << n):
            r = submask_rows(m, n)
            ref = leibniz_det(A[np.ix_(r, r)]) if r else 1.0
            assert abs(out[m] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, m, out[m], ref)


def pin_cminors_hermitian_pd(cminors):
    """Hermitian positive-definite => every principal minor is real and positive."""
    rng = _rng(22)
    n = 8
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = X @ X.conj().T + 0.5 * np.eye(n)
    out = cminors(H)
    assert np.all(out.real > 0)
    assert np.all(np.abs(out.imag) <= 1e-12 * np.abs(out.real))


def pin_cminors_det_I_plus_A(cminors):
    rng = _rng(23)
    n = 9
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    out = cminors(A)
    ref = np.linalg.det(np.eye(n) + A)
    assert abs(out.sum() - ref) <= 1e-10 * max(1.0, np.abs(out).sum())


def pin_cminors_conjugate(cminors):
    rng = _rng(24)
    n = 6
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    assert close(cminors(A.conj()), np.conj(cminors(A)), 1e-12, 1e-13)


CMINOR_PINS = [pin_cminors_leibniz, pin_cminors_hermitian_pd, pin_cminors_det_I_plus_A,
               pin_cminors_conjugate]


# ----------------------------------------------------------------------------------
# connected sums (Sec. V.A, Eq. (recursion))
# ----------------------------------------------------------------------------------
def _sizes(n):
    return np.array([bin(m).count("1") for m in range(1 << n)])


def pin_cs_factorial(cs):
    """a[S] = |S|!  =>  c[S] = (|S|-1)!  (number of permutations vs. number of cycles)."""
    n = 7
    sz = _sizes(n)
    a = np.array([math.factorial(k) for k in sz], dtype=np.float64)
    for mode in (0, 1):
        c = cs(a, mode)
        for m in range(1, 1 << n):
            if mode == 0 and not (m & 1):
                assert c[m] == 0.0
                continue
            assert c[m] == math.factorial(sz[m] - 1), (mode, m, c[m])


def pin_cs_diagonal(cs):
    """Multiplicative weights (diagonal M, a = prod d_i^2): c = 0 for |S| >= 2, c[{i}] = a[{i}]."""
    n = 8
    d = _rng(31).standard_normal(n)
    a = np.array([np.prod(d[submask_rows(m, n)] ** 2) for m in range(1 << n)])
    c = cs(a, 1)
    sz = _sizes(n)
    for m in range(1, 1 << n):
        if sz[m] == 1:
            assert c[m] == a[m]
        else:
            assert abs(c[m]) <= 1e-13 * max(1.0, np.abs(a).max()), (m, c[m])


def pin_cs_block_diag(cs):
    """Block-diagonal M: a factorises across blocks, so c vanishes on sets meeting both."""
    rng = _rng(32)
    n1, n2 = 3, 4
    n = n1 + n2
    A = np.zeros((n, n))
    A[:n1, :n1] = rng.standard_normal((n1, n1))
    A[n1:, n1:] = rng.standard_normal((n2, n2))
    a = np.array([leibniz_det(A[np.ix_(r, r)]) ** 2 if r else 1.0
                  for r in (submask_rows(m, n) for m in range(1 << n))])
    for mode in (0, 1):
        c = cs(a, mode)
        for m in range(1, 1 << n):
            if (m & ((1 << n1) - 1)) and (m >> n1):
                assert abs(c[m]) <= 1e-12 * max(1.0, abs(a[m])), (mode, m, c[m])


def pin_cs_exponential_formula(cs):
    """a[S] = sum over set partitions of S of prod_B c[B] (c from mode 1)."""
    n = 6
    a = np.empty(1 << n)
    rng = _rng(33)
    a[1:] = rng.standard_normal((1 << n) - 1)
    a[0] = 1.0
    c = cs(a, 1)
    for m in range(1, 1 << n):
        tot = 0.0
        for part in set_partitions(submask_rows(m, n)):
            prod = 1.0
            for blk in part:
                prod *= c[sum(1 << i for i in blk)]
            tot += prod
        assert abs(tot - a[m]) <= 1e-12 * max(1.0, np.abs(a).max()), (m, tot, a[m])


def pin_cs_root_independence(cs):
    """Any choice of the distinguished vertex gives the same c (Sec. V.A): relabel
    vertices in reverse so that 'lowest vertex' becomes 'highest vertex'."""
    n = 8
    rng = _rng(34)
    a = rng.standard_normal(1 << n)
    rev = np.array([int(format(m, f"0{n}b")[::-1], 2) for m in range(1 << n)])
    c = cs(a, 1)
    c_rev = cs(a[rev], 1)[rev]
    assert close(c_rev, c, 1e-10, 1e-12)


def pin_cs_single_det_cycles(cs):
    """a = det M (one determinant): c[S] = (-1)^(|S|-1) * sum over cyclic permutations
    of S of prod M_{i sigma(i)} (connected permutation diagrams are single cycles)."""
    n = 6
    M = _rng(35).standard_normal((n, n))
    a = np.array([leibniz_det(M[np.ix_(r, r)]) if r else 1.0
                  for r in (submask_rows(m, n) for m in range(1 << n))])
    c = cs(a, 1)
    for m in range(1, 1 << n):
        r = submask_rows(m, n)
        k = len(r)
        tot = 0.0
        for p in itertools.permutations(range(k)):
            # single k-cycle?
            j, L = 0, 0
            while True:
                j = p[j]
                L += 1
                if j == 0:
                    break
            if L != k:
                continue
            prod = 1.0
            for i in range(k):
                prod *= M[r[i], r[p[i]]]
            tot += prod
        ref = (-1) ** (k - 1) * tot
        assert abs(c[m] - ref) <= 1e-12 * max(1.0, abs(ref)), (m, c[m], ref)


CS_PINS = [pin_cs_factorial, pin_cs_diagonal, pin_cs_block_diag, pin_cs_exponential_formula,
           pin_cs_root_independence, pin_cs_single_det_cycles]


# ----------------------------------------------------------------------------------
# permanent principal minors (Sec. IV)
# ----------------------------------------------------------------------------------
def pin_perm_all_ones(perm):
    n = 7
    out = perm(np.ones((n, n)))
    for m in range(1 << n):
        assert out[m] == math.factorial(bin(m).count("1")), (m, out[m])


def pin_perm_diagonal(perm):
    d = _rng(41).standard_normal(6)
    out = perm(np.diag(d))
    for m in range(1 << 6):
        ref = np.prod(d[submask_rows(m, 6)])
        assert abs(out[m] - ref) <= 1e-14 * max(1.0, abs(ref))


def pin_perm_bruteforce(perm):
    rng = _rng(42)
    for n in (1, 2, 3, 5, 6):
        A = rng.standard_normal((n, n))
        out = perm(A)
        for m in range(1 << n):
            r = submask_rows(m, n)
            ref = brute_perm(A[np.ix_(r, r)]) if r else 1.0
            assert abs(out[m] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, m, out[m], ref)


def pin_perm_I_plus_A(perm):
    """sum_S per A[S] = per(I + A)."""
    n = 7
    A = _rng(43).standard_normal((n, n)) / np.sqrt(n)
    out = perm(A)
    ref = brute_perm(np.eye(n) + A)
    assert abs(out.sum() - ref) <= 1e-11 * max(1.0, np.abs(out).sum()), (out.sum(), ref)


def pin_perm_invariances(perm):
    n = 6
    rng = _rng(44)
    A = rng.standard_normal((n, n))
    out = perm(A)
    assert close(perm(A.T.copy()), out, 1e-12, 1e-13)
    p = rng.permutation(n)
    P = A[np.ix_(p, p)]
    outp = perm(P)
    # mask m of P <-> mask with bits p[k] of A
    mp = np.array([sum(1 << int(p[k]) for k in submask_rows(m, n)) for m in range(1 << n)])
    assert close(outp, out[mp], 1e-12, 1e-13)


PERM_PINS = [pin_perm_all_ones, pin_perm_diagonal, pin_perm_bruteforce, pin_perm_I_plus_A,
             pin_perm_invariances]


# ----------------------------------------------------------------------------------
# XOR minors of 2n x 2n block matrices (Sec. III, XOR case; Sec. V.C)
# ----------------------------------------------------------------------------------
def _xor_depth(out, k):
    return out[(1 << k) - 2:(1 << (k + 1)) - 2]


def _xor_rows(n, k, beta):
    """Rows of the depth-k entry beta: one row of each of the k trailing blocks."""
    return [2 * (n - k + i) + (beta >> i & 1) for i in range(k)]


def pin_xor_leibniz(xor):
    """Every entry against the permutation-sum determinant of its rows/columns."""
    rng = _rng(71)
    for n in (1, 2, 3):
        for cplx in (False, True):
            A = rng.standard_normal((2 * n, 2 * n))
            if cplx:
                A = A + 1j * rng.standard_normal((2 * n, 2 * n))
            out = xor(A)
            for k in range(1, n + 1):
                seg = _xor_depth(out, k)
                for alpha in range(1 << k):
                    r = _xor_rows(n, k, alpha)
                    ref = leibniz_det(A[np.ix_(r, r)])
                    assert abs(seg[alpha] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, k, alpha)


def pin_xor_block_diagonal(xor):
    """Zero blocks off the diagonal: each minor is the product of the kept diagonal entries."""
    rng = _rng(72)
    n = 6
    A = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    for i in range(n):
        A[2 * i:2 * i + 2, 2 * i:2 * i + 2] = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    out = xor(A)
    d = np.diag(A)
    for k in range(1, n + 1):
        seg = _xor_depth(out, k)
        ref = np.array([np.prod([d[r] for r in _xor_rows(n, k, a)]) for a in range(1 << k)])
        assert close(seg, ref, 1e-13, 1e-15), k


def pin_xor_branch_swap(xor):
    """Swapping the two rows/columns of every block maps choice alpha to its complement."""
    rng = _rng(73)
    n = 5
    A = rng.standard_normal((2 * n, 2 * n)) + 1j * rng.standard_normal((2 * n, 2 * n))
    perm = np.arange(2 * n) ^ 1
    out, out_s = xor(A), xor(A[np.ix_(perm, perm)])
    for k in range(1, n + 1):
        full = (1 << k) - 1
        seg, seg_s = _xor_depth(out, k), _xor_depth(out_s, k)
        assert close(seg_s, seg[np.arange(1 << k) ^ full], 1e-12, 1e-14), k


def pin_xor_largest_time(xor):
    """Keldysh block matrices: the row and column of the latest vertex do not depend on its
    branch, so the branch-signed sum of the determinants vanishes at every depth, while
    the unsigned sum does not."""
    from workloads import keldysh_block
    for b, A in enumerate(keldysh_block(3, 6, seed=74)):
        out = xor(A)
        for k in range(1, 7):
            seg = _xor_depth(out, k)
            sgn = np.array([(-1) ** bin(a).count("1") for a in range(1 << k)])
            scale = np.abs(seg).sum()
            assert scale > 0
            assert abs(np.dot(sgn, seg)) <= 1e-13 * scale, (b, k)
            assert abs(seg.sum()) > 1e-6 * scale or k == 1, (b, k)


def pin_xor_lapack(xor):
    """Order 5, every depth, against LAPACK's determinant of the gathered matrix."""
    rng = _rng(75)
    n = 5
    A = rng.standard_normal((2 * n, 2 * n)) + 1j * rng.standard_normal((2 * n, 2 * n))
    out = xor(A)
    for k in range(1, n + 1):
        seg = _xor_depth(out, k)
        ref = np.array([np.linalg.det(A[np.ix_(_xor_rows(n, k, a), _xor_rows(n, k, a))]) for a in range(1 << k)])
        assert close(seg, ref, 1e-12, 1e-13), k


XOR_PINS = [pin_xor_leibniz, pin_xor_block_diagonal, pin_xor_branch_swap, pin_xor_largest_time, pin_xor_lapack]


# ----------------------------------------------------------------------------------
# XNOR minors of 2n x 2n block matrices (Sec. III, XNOR case)
# ----------------------------------------------------------------------------------
def _xnor_rows(n, mask):
    return [r for i in range(n) if mask >> i & 1 for r in (2 * i, 2 * i + 1)]


def pin_xnor_leibniz(xnor):
    rng = _rng(81)
    for n in (1, 2, 3):
        for cplx in (False, True):
            A = rng.standard_normal((2 * n, 2 * n))
            if cplx:
                A = A + 1j * rng.standard_normal((2 * n, 2 * n))
            out = xnor(A)
            assert out[0] == 1.0
            for mask in range(1, 1 << n):
                r = _xnor_rows(n, mask)
                ref = leibniz_det(A[np.ix_(r, r)])
                assert abs(out[mask] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, mask)


def pin_xnor_block_diagonal(xnor):
    """Zero blocks off the diagonal: the product of the kept 2 x 2 determinants."""
    rng = _rng(82)
    n = 7
    A = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    d = []
    for i in range(n):
        blk = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        A[2 * i:2 * i + 2, 2 * i:2 * i + 2] = blk
        d.append(blk[0, 0] * blk[1, 1] - blk[0, 1] * blk[1, 0])
    out = xnor(A)
    ref = np.array([np.prod([d[i] for i in range(n) if m >> i & 1]) for m in range(1 << n)])
    assert close(out, ref, 1e-13, 1e-15)


def pin_xnor_block_similarity(xnor):
    """A -> D A D^-1 with D block diagonal (invertible 2 x 2 blocks) leaves every whole-block
    principal submatrix similar to the old one, so every XNOR minor is unchanged."""
    rng = _rng(83)
    n = 6
    A = rng.standard_normal((2 * n, 2 * n)) + 1j * rng.standard_normal((2 * n, 2 * n))
    D = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    for i in range(n):
        D[2 * i:2 * i + 2, 2 * i:2 * i + 2] = rng.standard_normal((2, 2)) + 2.0 * np.eye(2)
    out, out_s = xnor(A), xnor(D @ A @ np.linalg.inv(D))
    assert close(out_s, out, 1e-10, 1e-12)


def pin_xnor_lapack(xnor):
    rng = _rng(84)
    n = 5
    A = rng.standard_normal((2 * n, 2 * n))
    out = xnor(A)
    ref = np.array([np.linalg.det(A[np.ix_(_xnor_rows(n, m), _xnor_rows(n, m))]) if m else 1.0
                    for m in range(1 << n)])
    assert close(out, ref, 1e-12, 1e-13)


XNOR_PINS = [pin_xnor_leibniz, pin_xnor_block_diagonal, pin_xnor_block_similarity, pin_xnor_lapack]


# ----------------------------------------------------------------------------------
# leading principal minors (Sec. III)
# ----------------------------------------------------------------------------------
def pin_lead_triangular(lead):
    """Lower triangular: the running products of the diagonal."""
    rng = _rng(91)
    n = 12
    A = np.tril(rng.standard_normal((n, n))) + 1j * np.tril(rng.standard_normal((n, n)))
    assert close(lead(A), np.cumprod(np.diag(A)), 1e-13, 1e-15)


def pin_lead_leibniz(lead):
    rng = _rng(92)
    for n in (1, 2, 3, 5):
        A = rng.standard_normal((n, n))
        out = lead(A)
        for k in range(1, n + 1):
            ref = leibniz_det(A[:k, :k])
            assert abs(out[k - 1] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, k)


def pin_lead_ratio(lead):
    """det A[:k,:k] / det A[:k-1,:k-1] is the last pivot of elimination without row
    exchanges, i.e. 1 / (A[:k,:k]^-1)[k-1, k-1] (Cramer's rule)."""
    rng = _rng(93)
    n = 9
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 3 * np.eye(n)
    out = lead(A)
    for k in range(2, n + 1):
        piv = 1.0 / np.linalg.inv(A[:k, :k])[k - 1, k - 1]
        assert abs(out[k - 1] / out[k - 2] - piv) <= 1e-11 * abs(piv), k


LEAD_PINS = [pin_lead_triangular, pin_lead_leibniz, pin_lead_ratio]


# ----------------------------------------------------------------------------------
# NAND minors of 2n x 2n block matrices (Sec. III, NAND case)
# ----------------------------------------------------------------------------------
def _nand_rows(n, code):
    r = []
    for i in range(n):
        t = code % 3
        code //= 3
        if t:
            r.append(2 * i + t - 1)
    return r


def pin_nand_leibniz(nand):
    rng = _rng(101)
    for n in (1, 2, 3):
        for cplx in (False, True):
            A = rng.standard_normal((2 * n, 2 * n))
            if cplx:
                A = A + 1j * rng.standard_normal((2 * n, 2 * n))
            out = nand(A)
            assert out[0] == 1.0
            for code in range(1, 3 ** n):
                r = _nand_rows(n, code)
                ref = leibniz_det(A[np.ix_(r, r)])
                assert abs(out[code] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, code)


def pin_nand_contains_xor(nand):
    """The entries with no block left out are the order-n XOR minors (Sec. III): choice
    word beta maps to code sum_i (beta_i + 1) 3^i; they are the polynomial matrix's top
    coefficients in the paper's alpha reading, checked here against determinants."""
    rng = _rng(102)
    n = 5
    A = rng.standard_normal((2 * n, 2 * n)) + 1j * rng.standard_normal((2 * n, 2 * n))
    out = nand(A)
    for beta in range(1 << n):
        code = sum(((beta >> i & 1) + 1) * 3 ** i for i in range(n))
        r = [2 * i + (beta >> i & 1) for i in range(n)]
        ref = np.linalg.det(A[np.ix_(r, r)])
        assert abs(out[code] - ref) <= 1e-11 * max(1.0, abs(ref)), beta


def pin_nand_block_diagonal(nand):
    """Zero off-diagonal blocks and diagonal 2 x 2 blocks: each minor is the product of the
    kept diagonal entries."""
    rng = _rng(103)
    n = 6
    A = np.zeros((2 * n, 2 * n))
    for i in range(n):
        A[2 * i:2 * i + 2, 2 * i:2 * i + 2] = rng.standard_normal((2, 2))
    out = nand(A)
    d = np.diag(A)
    ref = np.array([np.prod([d[r] for r in _nand_rows(n, c)]) for c in range(3 ** n)])
    assert close(out, ref, 1e-13, 1e-15)


def pin_nand_sum(nand):
    """With every off-diagonal block zero, the sum of all NAND minors factorises into
    prod_i (1 + A[2i, 2i] + A[2i+1, 2i+1]) (each block contributes nothing or one of its
    two diagonal entries)."""
    rng = _rng(104)
    n = 7
    A = np.zeros((2 * n, 2 * n))
    for i in range(n):
        A[2 * i:2 * i + 2, 2 * i:2 * i + 2] = rng.standard_normal((2, 2))
    out = nand(A)
    ref = np.prod([1 + A[2 * i, 2 * i] + A[2 * i + 1, 2 * i + 1] for i in range(n)])
    assert abs(out.sum() - ref) <= 1e-12 * max(1.0, abs(ref))


NAND_PINS = [pin_nand_leibniz, pin_nand_contains_xor, pin_nand_block_diagonal, pin_nand_sum]
