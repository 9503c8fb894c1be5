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
