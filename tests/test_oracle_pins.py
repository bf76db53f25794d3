"""CPU pins of the oracle (no GPU): hand-worked golden cases, brute force,
closed forms, invariants and special cases; plus planted-mistake builds of the
oracle that every pin set must reject."""

import os
import tempfile

import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def ora():
    return oracle.get()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(ora, pin):
    pin(ora)


# Planted mistakes, each a plausible slip in the oracle's arithmetic:
#  1 open instead of closed boundaries      2 x/y transposed in one compare
#  3 one compare dropped                     4 parent MBR loses the max-x union
#  5 STR drops the last item of each slice   6 ids left unsorted
#  7 pair sides swapped in the leaf-vs-subtree join case
#  8 many-to-many update moves the gather index the wrong way on a clear bit
#  9 outer slicing (O3) treats touching children as disjoint
# 10 the tree checker skips the parent-MBR == union-of-children comparison
# 11 the tree checker skips the child-level comparison
MUTANTS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11]


@pytest.mark.parametrize("mutant", MUTANTS)
def test_pins_catch_mutant(mutant):
    d = tempfile.mkdtemp(prefix="ora_mut_")
    path = os.path.join(d, f"liboracle_m{mutant}.so")
    oracle.build(path, mutant=mutant)
    bad = oracle.Oracle(path)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(bad)
        except (AssertionError, ValueError) as e:  # noqa: PERF203
            caught.append(pin.__name__)
    assert caught, f"mutant {mutant} passed every pin"
