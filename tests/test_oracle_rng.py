"""Pins of the oracle's counter-based generator (SplitMix64)."""
import os

import numpy as np

from oracle import rng

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_published_outputs():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    for idx, hexval in rows:
        assert rng.sm(0, int(idx)) == int(hexval, 16)


def test_vectorised_matches_scalar():
    seeds = [0, 1, 2 ** 63 + 12345, 2 ** 64 - 1]
    ns = np.array([0, 1, 7, 1000, 2 ** 40 + 3], dtype=np.uint64)
    for s in seeds:
        v = rng.sm_vec(s, ns)
        for n, x in zip(ns, v):
            assert int(x) == rng.sm(s, int(n))


def test_u53_and_below_ranges():
    xs = [0, 1, 2 ** 11 - 1, 2 ** 11, 2 ** 64 - 1, rng.sm(3, 4)]
    for x in xs:
        u = rng.u53(x)
        assert 0.0 <= u < 1.0
        assert u == (x >> 11) / 2.0 ** 53
        for n in (1, 2, 3, 20000, 2 ** 31 - 1):
            b = rng.below(x, n)
            assert 0 <= b < n
            # floor(x * n / 2**64) by exact rational comparison
            assert b * 2 ** 64 <= x * n < (b + 1) * 2 ** 64
