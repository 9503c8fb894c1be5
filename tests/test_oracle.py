"""The CPU oracle against facts the paper and mathematics fix (no GPU needed)."""
import math

import numpy as np
import pytest

import oracle_pins as P
import workloads as W


@pytest.mark.parametrize("pin", P.MINOR_PINS, ids=lambda f: f.__name__)
def test_minor_pins(oracle_mod, pin):
    pin(oracle_mod.minors)


@pytest.mark.parametrize("pin", P.CMINOR_PINS, ids=lambda f: f.__name__)
def test_complex_minor_pins(oracle_mod, pin):
    pin(oracle_mod.minors_complex)


@pytest.mark.parametrize("pin", P.CS_PINS, ids=lambda f: f.__name__)
def test_connected_sum_pins(oracle_mod, pin):
    pin(lambda a, mode: oracle_mod.connected_sums(a, mode))


@pytest.mark.parametrize("pin", P.PERM_PINS, ids=lambda f: f.__name__)
def test_perm_pins(oracle_mod, pin):
    pin(oracle_mod.perm_minors)


@pytest.mark.parametrize("pin", P.NAND_PINS, ids=lambda f: f.__name__)
def test_nand_minor_pins(oracle_mod, pin):
    pin(oracle_mod.nand_minors)


@pytest.mark.parametrize("pin", P.LEAD_PINS, ids=lambda f: f.__name__)
def test_leading_minor_pins(oracle_mod, pin):
    pin(oracle_mod.leading_minors)


@pytest.mark.parametrize("pin", P.XNOR_PINS, ids=lambda f: f.__name__)
def test_xnor_minor_pins(oracle_mod, pin):
    pin(oracle_mod.xnor_minors)


@pytest.mark.parametrize("pin", P.XOR_PINS, ids=lambda f: f.__name__)
def test_xor_minor_pins(oracle_mod, pin):
    pin(oracle_mod.xor_minors)


@pytest.mark.parametrize("pin", P.PERM_PINS, ids=lambda f: f.__name__)
def test_perm_masks_pins(oracle_mod, pin):
    """The mask-list entry point (used to sample large orders) meets the same pins."""
    pin(lambda A: oracle_mod.perm_minors_at(A, np.arange(1 << np.asarray(A).shape[0], dtype=np.uint32)))


def test_ragged_matches_uniform(oracle_mod):
    rng = np.random.default_rng(5)
    mats = [rng.standard_normal((k, k)) for k in (3, 1, 6, 4)]
    outs = oracle_mod.minors_ragged(mats)
    for M, o in zip(mats, outs):
        np.testing.assert_array_equal(o, oracle_mod.minors(M))


def test_rooted_mode_zero_outside_root(oracle_mod):
    a = np.random.default_rng(6).standard_normal(1 << 6)
    c0 = oracle_mod.connected_sums(a, 0)
    c1 = oracle_mod.connected_sums(a, 1)
    for m in range(1, 1 << 6):
        if m & 1:
            assert c0[m] == c1[m]       # the lowest vertex of a set containing 0 is 0
        else:
            assert c0[m] == 0.0


def test_cs_input_bound_bounds_perturbations(oracle_mod):
    """The first-order error bound of the recursion covers actual perturbations of a."""
    rng = np.random.default_rng(17)
    n = 7
    for mode in (0, 1):
        a = rng.standard_normal(1 << n)
        c = oracle_mod.connected_sums(a, mode)
        da = np.abs(a) * 1e-9 + 1e-12
        e = oracle_mod.cs_input_bound(a, c, da, mode)
        worst = 0.0
        for _ in range(20):
            pert = a + da * rng.uniform(-1, 1, a.shape)
            diff = np.abs(oracle_mod.connected_sums(pert, mode) - c)
            worst = max(worst, float(np.max(diff / (e + 1e-300))))
        assert worst <= 1.0 + 1e-6
        # and a single-entry perturbation at the full bound is reached exactly at first order
        S = (1 << n) - 1
        p2 = a.copy()
        p2[S] += da[S]
        assert abs(oracle_mod.connected_sums(p2, mode)[S] - c[S]) <= e[S] * (1 + 1e-6)


def test_hadamard_batch_matches_single():
    from oracle import metrics
    A = np.random.default_rng(3).standard_normal((4, 6, 6))
    Hb = metrics.hadamard_bounds_batch(A)
    for b in range(4):
        np.testing.assert_allclose(Hb[b], metrics.hadamard_bounds(A[b]), rtol=1e-14)


@pytest.mark.parametrize("pin", P.MINOR_PINS, ids=lambda f: f.__name__)
def test_minor_masks_pins(oracle_mod, pin):
    """The mask-list entry point (the reference for every order above 14 and for the
    sampled full-size batches) meets the same pins as the all-masks routine."""
    pin(lambda A: P.minors_via_masks(oracle_mod, A))


# ---- the error metrics that set every gate, pinned to facts outside themselves ------------

def test_hadamard_at_matches_hadamard_bounds():
    """Two separate evaluations of H_S = prod_{i in S} ||A[i, S]||_2: prefix sums of the
    squared rows in log space (all masks) and explicit norms (listed masks)."""
    from oracle import metrics
    rng = np.random.default_rng(41)
    for n in (1, 4, 7):
        A = rng.standard_normal((n, n)) * rng.uniform(0.01, 10, (n, 1))
        H = metrics.hadamard_bounds(A)
        masks = np.arange(1 << n)
        np.testing.assert_allclose(metrics.hadamard_at(A, masks), H, rtol=1e-13)
        assert H[0] == 1.0
    # entries whose squares overflow or underflow fp64 (numpy's norm rescales internally)
    A = rng.standard_normal((6, 6)) * np.array([2.0 ** 600, 1.0, 2.0 ** -560, 1.0, 1.0, 1.0])[:, None]
    H = metrics.hadamard_bounds(A)
    assert np.all(np.isfinite(H[1:])) and np.all(H[1:] > 0)
    np.testing.assert_allclose(metrics.hadamard_at(A, np.arange(64)), H, rtol=1e-13)
    np.testing.assert_allclose(metrics.hadamard_bounds_batch(A[None])[0], H, rtol=1e-14)


def test_hadamard_inequality_and_equality():
    """Hadamard's inequality |det M| <= prod_i ||M[i, :]||_2 for every principal submatrix
    (determinants from numpy's LAPACK, not from the oracle), with equality when the rows
    are orthogonal: for every subset of a diagonal matrix, and for the full set of a
    matrix with orthogonal rows."""
    from oracle import metrics
    rng = np.random.default_rng(42)
    n = 7
    for _ in range(3):
        A = rng.standard_normal((n, n))
        H = metrics.hadamard_bounds(A)
        for m in range(1, 1 << n):
            r = [k for k in range(n) if m >> k & 1]
            d = np.linalg.det(A[np.ix_(r, r)])
            assert abs(d) <= H[m] * (1 + 1e-12), (m, d, H[m])
    D = np.diag(rng.uniform(-3, 3, n))
    H = metrics.hadamard_bounds(D)
    for m in range(1 << n):
        r = [k for k in range(n) if m >> k & 1]
        assert abs(abs(np.prod(np.diag(D)[r])) - H[m]) <= 1e-14 * H[m]
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q * rng.uniform(0.5, 2.0, (n, 1))               # orthogonal rows of chosen lengths
    H = metrics.hadamard_bounds(A)
    assert abs(abs(np.linalg.det(A)) - H[-1]) <= 1e-13 * H[-1]


def test_mixed_err_definition():
    """e = |x - ref| / max(|ref|, H): zero for equal values (also both zero), relative
    error where |ref| dominates, error relative to H where the minor is (near) zero, and
    infinite for a non-finite value against a finite reference."""
    from oracle import metrics
    e = metrics.mixed_err(np.array([1.0, 0.0, 2.0 + 1e-6, 1e-3, np.nan]),
                          np.array([1.0, 0.0, 2.0, 0.0, 1.0]),
                          np.array([1.5, 0.0, 1.0, 10.0, 1.0]))
    assert e[0] == 0.0 and e[1] == 0.0
    assert abs(e[2] - 0.5e-6) <= 1e-9 * 0.5e-6      # (2 + 1e-6) - 2 is 1e-6 to fp64 rounding
    assert abs(e[3] - 1e-4) <= 1e-15 * 1e-4
    assert np.isinf(e[4])


def _closed_form_weights(n):
    return np.array([math.factorial(bin(S).count("1")) if S else 0.0 for S in range(1 << n)])


@pytest.mark.parametrize("mode", [0, 1])
def test_cs_scale_closed_form(oracle_mod, mode):
    """For a[S] = |S|! the recursion gives c[S] = (|S| - 1)!, so its scale has the closed
    form d[S] = |S|! + sum_{t=1}^{k-1} C(k-1, t-1) (t-1)! (k-t)! = (k-1)! (2k - 1), k = |S|
    (the terms c[T] a[S \\ T] of Eq. (recursion) summed in magnitude)."""
    n = 7
    a = _closed_form_weights(n)
    c = oracle_mod.connected_sums(a, mode)
    d = oracle_mod.cs_scale(a, c, mode)
    for S in range(1, 1 << n):
        if mode == 0 and not S & 1:
            assert d[S] == 0.0
            continue
        k = bin(S).count("1")
        assert d[S] == math.factorial(k - 1) * (2 * k - 1), (S, d[S])


@pytest.mark.parametrize("mode", [0, 1])
def test_cs_scale_bounds_rounding(oracle_mod, mode):
    """d[S] is the scale of the recursion's rounding: the fp64 connected sums differ from
    the same recursion evaluated exactly in rational arithmetic (Python fractions) by at
    most a small multiple of eps * d[S], and |c[S]| <= d[S] always."""
    from fractions import Fraction
    n = 6
    rng = np.random.default_rng(43)
    a = rng.standard_normal(1 << n)
    c = oracle_mod.connected_sums(a, mode)
    d = oracle_mod.cs_scale(a, c, mode)
    assert np.all(np.abs(c) <= d * (1 + 1e-15))
    fa = [Fraction(float(x)) for x in a]
    fc = [Fraction(0)] * (1 << n)
    for S in range(1, 1 << n):
        j = 1 if mode == 0 else (S & -S)
        if not S & j:
            continue
        acc = fa[S]
        for T in range(1, S):
            if T & S == T and T & j:
                acc -= fc[T] * fa[S & ~T]
        fc[S] = acc
    eps = np.finfo(float).eps
    worst = max(abs(float(Fraction(float(c[S])) - fc[S])) / (eps * d[S]) for S in range(1, 1 << n) if d[S] > 0)
    assert worst <= 2.0 * n, worst


def test_cdet_tolerance_covers_minor_errors(oracle_mod):
    """The connected-sum tolerance used when the weights come from independently rounded
    minors: perturbing every minor by up to eps_minor * max(|m|, H_S) (the minors' own
    gate) moves the connected sums by no more than the tolerance; with eps_minor = 0 it
    is eps_cs times the recursion scale."""
    from oracle import metrics
    rng = np.random.default_rng(44)
    A = W.lattice_batch(3, 7, W.Lattice(8, 1.0, 0.0, 2.0), seed=44)
    m = oracle_mod.minors(A)
    c = oracle_mod.connected_sums(m * m, 0)
    tol = metrics.cdet_tolerance(A, m, c, eps_minor=1e-6, eps_cs=0.0)
    H = metrics.hadamard_bounds_batch(A)
    for _ in range(10):
        dm = 1e-6 * np.maximum(np.abs(m), H) * rng.uniform(-1, 1, m.shape)
        dm[:, 0] = 0.0
        mp = m + dm
        cp = oracle_mod.connected_sums(mp * mp, 0)
        assert np.all(np.abs(cp - c) <= tol * (1 + 1e-6) + 1e-300)
    tol0 = metrics.cdet_tolerance(A, m, c, eps_minor=0.0, eps_cs=1e-10)
    np.testing.assert_allclose(tol0, 1e-10 * oracle_mod.cs_scale(m * m, c, 0), rtol=1e-15)
