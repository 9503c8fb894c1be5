"""The CPU oracle against facts the paper and mathematics fix (no GPU needed)."""
import numpy as np
import pytest

import oracle_pins as P


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
