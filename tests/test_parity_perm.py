"""GPU parity of apm_all_perm_minors (Sec. IV) against the CPU oracle (per-subset Ryser).

Gate: |x - ref| <= 1e-10 * sum_{T subset of S} |prod_{i in S} r_i(T)| + tiny, i.e. relative to
the magnitude of the inclusion-exclusion terms (the formula's own rounding scale); the
scale is bounded here by prod_{i in S} sum_j |A_ij| * 2^|S|."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def apm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_07638_amd as m
    return m


def scale(A):
    n = A.shape[0]
    rs = np.abs(A).sum(axis=1)
    out = np.empty(1 << n)
    for s in range(1 << n):
        idx = [i for i in range(n) if s >> i & 1]
        out[s] = np.prod(rs[idx]) * (2.0 ** len(idx))
    return out


def run(apm, A):
    import torch
    got = apm.all_perm_minors(torch.from_numpy(np.ascontiguousarray(A)).cuda())
    torch.cuda.synchronize()
    return got.cpu().numpy()


@pytest.mark.parametrize("n", list(range(1, 13)) + [14])
def test_gauss_orders(apm, oracle_mod, n):
    A = W.gauss_batch(3, n, seed=200 + n)
    got = run(apm, A)
    ref = oracle_mod.perm_minors(A)
    for b in range(3):
        assert np.all(np.abs(got[b] - ref[b]) <= TOL * scale(A[b])), n


def test_gauss_order_13(apm, oracle_mod):
    """Orders above 12 split their highest indices over workgroups (one per subset of them)."""
    A = W.gauss_batch(1, 13, seed=413)
    got = run(apm, A)
    ref = oracle_mod.perm_minors(A)
    assert np.all(np.abs(got[0] - ref[0]) <= TOL * scale(A[0]))


@pytest.mark.parametrize("n", [15, 16])
def test_gauss_large_orders_sampled(apm, oracle_mod, n):
    """Sampled subsets at the largest orders: every subset of the workgroup-split indices
    (each workgroup's full set), the full set, and random subsets."""
    A = W.gauss_batch(2, n, seed=400 + n)
    got = run(apm, A)
    rng = np.random.default_rng(n)
    hi = [(m << 12) | 0xFFF for m in range(1 << (n - 12))]
    masks = np.unique(np.concatenate([np.array(hi, dtype=np.uint32),
                                      rng.integers(0, 1 << n, 64, dtype=np.uint32),
                                      np.array([0, (1 << n) - 1], dtype=np.uint32)]))
    for b in range(2):
        ref = oracle_mod.perm_minors_at(A[b], masks)
        sc = scale(A[b])[masks]
        assert np.all(np.abs(got[b][masks] - ref) <= TOL * sc), n


def test_all_ones_factorials(apm):
    n = 10
    got = run(apm, np.ones((1, n, n)))[0]
    for s in range(1 << n):
        assert got[s] == math.factorial(bin(s).count("1"))


def test_sum_is_per_of_I_plus_A(apm):
    """sum_S per(A[S]) = per(I + A), brute force over permutations for n = 7."""
    import itertools
    n = 7
    A = W.gauss_batch(1, n, seed=77)[0]
    got = run(apm, A[None])[0]
    M = np.eye(n) + A
    ref = sum(np.prod([M[i, p[i]] for i in range(n)]) for p in itertools.permutations(range(n)))
    assert abs(got.sum() - ref) <= 1e-10 * np.abs(got).sum()
