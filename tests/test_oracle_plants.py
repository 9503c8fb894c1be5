"""The pins have power: each plausible mistake planted in the oracle (a wrong sign,
index or operand; a dropped term) makes at least one pin fail.  Planted variants
are built from the oracle's own source on the CPU with -DORACLE_PLANT=k."""
import os
import tempfile

import pytest

import oracle_pins as P

PLANTS = {
    1: ("minors", "row-swap sign dropped"),
    2: ("minors", "transposed operand in the elimination update"),
    3: ("cs", "a[T] used instead of a[S \\ T]"),
    4: ("cs", "extra term: root singleton counted twice"),
    5: ("perm", "Ryser sign without the (-1)^|S| factor"),
    6: ("cminors", "conjugated quotient in the complex elimination"),
    7: ("xor", "the other row of every block kept"),
    8: ("xor", "columns taken from the other branch of each block"),
    9: ("xnor", "the first row of a kept block taken twice"),
    10: ("lead", "entry k holds the leading minor of order k - 1"),
    11: ("nand", "the two kept-row choices of a block swapped"),
    12: ("minors_at", "mask bits read in reversed order by the mask-list gather"),
    13: ("minors_at", "the last kept row gathered twice by the mask-list gather"),
}


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_mistake_is_caught(oracle_mod, plant):
    kind, what = PLANTS[plant]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, f"liboracle_plant{plant}.so")
        oracle_mod.build(force=True, path=path, plant=plant)
        lib = oracle_mod.load_library(path)
        if kind == "minors":
            fn, pins = (lambda A: oracle_mod.minors(A, lib=lib)), P.MINOR_PINS
        elif kind == "minors_at":
            fn, pins = (lambda A: P.minors_via_masks(oracle_mod, A, lib=lib)), P.MINOR_PINS
        elif kind == "cminors":
            fn, pins = (lambda A: oracle_mod.minors_complex(A, lib=lib)), P.CMINOR_PINS
        elif kind == "nand":
            fn, pins = (lambda A: oracle_mod.nand_minors(A, lib=lib)), P.NAND_PINS
        elif kind == "lead":
            fn, pins = (lambda A: oracle_mod.leading_minors(A, lib=lib)), P.LEAD_PINS
        elif kind == "xnor":
            fn, pins = (lambda A: oracle_mod.xnor_minors(A, lib=lib)), P.XNOR_PINS
        elif kind == "xor":
            fn, pins = (lambda A: oracle_mod.xor_minors(A, lib=lib)), P.XOR_PINS
        elif kind == "cs":
            fn, pins = (lambda a, mode: oracle_mod.connected_sums(a, mode, lib=lib)), P.CS_PINS
        else:
            fn, pins = (lambda A: oracle_mod.perm_minors(A, lib=lib)), P.PERM_PINS
        failed = []
        for pin in pins:
            try:
                pin(fn)
            except AssertionError:
                failed.append(pin.__name__)
        assert failed, f"no pin caught planted mistake {plant}: {what}"
