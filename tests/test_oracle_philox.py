"""Pins of the oracle's counter RNG and 128-bit multiply (CPU only)."""
import os
import random

import numpy as np
import pytest

import oracle as O
from oracle.philox_ref import philox4x32

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_philox_known_answers_c(ctr, key, want):
    assert O.philox(key, ctr) == want


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_philox_known_answers_python(ctr, key, want):
    assert philox4x32(key, ctr) == want


def test_philox_two_implementations_agree():
    rng = random.Random(1234)
    for _ in range(3000):
        key = [rng.getrandbits(32) for _ in range(2)]
        ctr = [rng.getrandbits(32) for _ in range(4)]
        assert O.philox(key, ctr) == philox4x32(key, ctr)


def test_philox_round_count_matters():
    # a generator with fewer rounds must not pass: guards against a loop bound slip
    key, ctr = [0, 0], [0, 0, 0, 0]
    assert philox4x32(key, ctr, rounds=9) != O.philox(key, ctr)


def test_philox_bit_balance():
    # each output bit is set about half the time over consecutive counters
    bits = np.zeros(128)
    N = 4000
    for i in range(N):
        r = O.philox([7, 9], [i, 0, 0, 0])
        for w in range(4):
            for b in range(32):
                bits[w * 32 + b] += (r[w] >> b) & 1
    frac = bits / N
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / np.sqrt(N))


def test_hi64_matches_big_integers():
    rng = random.Random(5)
    edge = [0, 1, 2, (1 << 32) - 1, 1 << 32, (1 << 63), (1 << 64) - 1]
    vals = edge + [rng.getrandbits(64) for _ in range(500)]
    for x in vals[:60]:
        for y in vals[:60]:
            assert O.hi64(x, y) == (x * y) >> 64
