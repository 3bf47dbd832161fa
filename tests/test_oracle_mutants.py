"""The pins must catch plausible mistakes: each planted mistake (a copy of the
oracle built with -DORACLE_MUTANT=n, CPU only) fails at least one pin."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle.build import build_mutant

import test_oracle_pins as pins
import bruteforce as bf

MUTANTS = {1: "'>=' instead of '>'", 2: "sample std", 3: "ties round up", 4: "upper median",
           5: "wrong bin mean", 6: "raw-column statistics in FD", 7: "wrong bin replaced",
           8: "last sample skipped", 9: "set-aside samples in masked statistics",
           10: "mask not cleared at a new run of masked steps"}


def _agrees_with_bruteforce(lib) -> bool:
    for seed in range(60):
        rng = np.random.default_rng(5000 + seed)
        C, T = int(rng.integers(2, 9)), int(rng.integers(2, 13))
        x = (rng.integers(0, int(rng.choice([2, 8, 256])), size=(C, T)).astype(np.uint8)
             if seed % 2 == 0 else pins.rand_f32(rng, (C, T)))
        steps = pins.rand_steps(rng, C, int(rng.integers(1, 4)))
        want, wbits = bf.pipeline(x, steps)
        got, gbits = oracle.pipeline(x, steps, want_flags=True, _lib_override=lib)
        if not (np.array_equal(got.view(np.uint8), want.view(np.uint8)) and np.array_equal(gbits, wbits)):
            return False
    for seed in range(40):
        rng = np.random.default_rng(8000 + seed)
        C, T = int(rng.integers(1, 6)), int(rng.integers(2, 13))
        x = rng.integers(0, int(rng.choice([2, 8, 256])), size=(C, T)).astype(np.uint8)
        steps = pins.rand_steps(rng, C, int(rng.integers(2, 6)), masked=True)
        want, wbits = bf.pipeline(x, steps)
        got, gbits = oracle.pipeline(x, steps, want_flags=True, _lib_override=lib)
        if not (np.array_equal(got, want) and np.array_equal(gbits, wbits)):
            return False
    # hand cases and closed forms: row [0 x9, 25] has mean 2.5 and the 25 sits
    # exactly 3 sigma out, so at k = 2.75 it is replaced by round(2.5) = 2
    x = np.array([[0] * 9 + [25]], np.uint8)
    got, _ = oracle.pipeline(x, [("td", 2.75, "mean", 0)], True, _lib_override=lib)
    if got[0, 9] != 2:
        return False
    for n, k in ((10, 3.0), (17, 4.0), (11, 3.0), (18, 4.0)):
        x = np.zeros((1, n), np.uint8)
        x[0, 0] = 5
        _, fl = oracle.pipeline(x, [("td", k, "mean", 0)], True, _lib_override=lib)
        if bool(fl[0, 0]) != (n - 1 > k * k):
            return False
    return True


@pytest.mark.parametrize("n", sorted(MUTANTS))
def test_planted_mistake_is_caught(n, tmp_path):
    lib = oracle._bind(build_mutant(n, str(tmp_path / f"mutant{n}.so")))
    assert not _agrees_with_bruteforce(lib), f"pins missed mutant {n}: {MUTANTS[n]}"


def test_unmutated_oracle_passes_the_same_check():
    assert _agrees_with_bruteforce(oracle._load())
