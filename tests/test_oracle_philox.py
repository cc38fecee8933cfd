"""Pins of the oracle's Philox4x32-10 and of its (0,1) uniform.

Philox4x32-10 is pinned to the published known-answer vectors of Salmon et al.
(SC'11), stored with their citation in tests/golden/philox4x32_10_kat.txt.
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(oracle_mod, ctr, key, expect):
    assert list(oracle_mod.philox4x32_10(ctr, key)) == expect


def test_u52_range_and_exactness(oracle_mod):
    u = oracle_mod.u52
    assert u(0, 0) == 2.0 ** -53
    assert u(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    # the low 12 bits of the 64-bit word are dropped
    assert u(0xFFF, 0) == u(0, 0)
    assert u(0x1000, 0) == 3.0 * 2.0 ** -53
    # midpoint
    assert u(0, 0x80000000) == 0.5 + 2.0 ** -53


def test_u52_uniformity(oracle_mod):
    rng = np.random.default_rng(7)
    words = rng.integers(0, 2 ** 32, size=(20000, 2), dtype=np.uint64)
    us = np.array([oracle_mod.u52(int(a), int(b)) for a, b in words])
    assert np.all((us > 0) & (us < 1))
    # mean and variance of U(0,1) within 5 sigma
    n = len(us)
    assert abs(us.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(us.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)


def test_philox_counter_sensitivity(oracle_mod):
    """Every counter and key word changes the output (no dropped input word)."""
    base_c, base_k = [1, 2, 3, 4], [5, 6]
    ref = oracle_mod.philox4x32_10(base_c, base_k)
    for i in range(4):
        c = list(base_c)
        c[i] ^= 1
        assert oracle_mod.philox4x32_10(c, base_k) != ref
    for i in range(2):
        k = list(base_k)
        k[i] ^= 1
        assert oracle_mod.philox4x32_10(base_c, k) != ref
