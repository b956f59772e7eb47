"""Pins of the counter-based draws (SplitMix64 published outputs)."""
import os

import pytest

from oracle.rng import (counter, draw_a, draw_b, draw_beta, draw_sigma, inverse_mod,
                        splitmix64)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_vectors.txt")


def golden_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        s, c, v = line.split()
        rows.append((int(s), int(c), int(v, 16)))
    return rows


@pytest.mark.parametrize("seed,c,expect", golden_rows())
def test_splitmix64_reference_outputs(seed, c, expect):
    assert splitmix64(seed, c) == expect


def test_draw_ranges_and_inverse():
    for n in (1 << 4, 1 << 14, 1 << 22, 1 << 26):
        for r in range(20):
            s = draw_sigma(99, n, r)
            assert s % 2 == 1 and 0 < s < n
            assert (s * inverse_mod(s, n)) % n == 1
            assert 0 <= draw_b(99, n, r) < n
            assert 0 <= draw_a(99, n, r, 1, 2) < n
            lo, hi = 17, 33
            assert lo <= draw_beta(99, lo, hi, r, 1, 0) <= hi


def test_counter_fields_do_not_overlap():
    seen = set()
    for r in range(3):
        for lev in (0, 1, 7, 0xFFF):
            for rep in range(4):
                for p in range(1, 5):
                    c = counter(r, lev, rep, p)
                    assert c not in seen
                    seen.add(c)
