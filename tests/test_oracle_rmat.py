"""Pins of the oracle's R-MAT generator and CSR construction (CPU only)."""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle as O


def test_thresholds_are_rounded_cumulative_probabilities():
    for a, b, c in [(0.57, 0.19, 0.19), (0.65, 0.15, 0.15), (0.25, 0.25, 0.25), (0.18, 0.25, 0.25)]:
        want = []
        for x in (Fraction(a), Fraction(a) + Fraction(b), Fraction(a) + Fraction(b) + Fraction(c)):
            want.append(round(x * (1 << 32)))
        got = O.rmat_thresholds(a, b, c)
        # the oracle rounds in double precision; the exact rational rounding agrees here
        assert got == want


def test_thresholds_known_values():
    assert O.rmat_thresholds(0.57, 0.19, 0.19) == [2448131359, 3264175145, 4080218931]
    assert O.rmat_thresholds(0.65, 0.15, 0.15) == [2791728742, 3435973837, 4080218931]


@pytest.mark.parametrize("abc", [(0.57, 0.19, 0.19), (0.65, 0.15, 0.15)])
def test_quadrant_frequencies_every_level(abc):
    a, b, c = abc
    d = 1.0 - a - b - c
    S = 12
    N = 100_000
    u, v = O.rmat_raw(S, a, b, c, 99, 0, N)
    for lvl in range(S):
        bit = S - 1 - lvl
        quad = (((u >> bit) & 1) << 1) | ((v >> bit) & 1)
        obs = np.bincount(quad.astype(np.int64), minlength=4)
        exp = N * np.array([a, b, c, d])
        p = stats.chisquare(obs, exp).pvalue
        assert p > 1e-5, (lvl, obs, exp)


def test_row_zero_expectation():
    # P(u == 0) = (a+b)^S: every level must pick a top quadrant
    a, b, c = 0.57, 0.19, 0.19
    S, N = 10, 400_000
    u, v = O.rmat_raw(S, a, b, c, 3, 0, N)
    for ids, pz in ((u, (a + b) ** S), (v, (a + c) ** S)):
        k = int(np.sum(ids == 0))
        mu, sd = N * pz, np.sqrt(N * pz * (1 - pz))
        assert abs(k - mu) < 5 * sd, (k, mu, sd)


def test_edge_is_pure_function_of_seed_and_index():
    u1, v1 = O.rmat_raw(14, 0.57, 0.19, 0.19, 5, 1000, 64)
    u2, v2 = O.rmat_raw(14, 0.57, 0.19, 0.19, 5, 0, 1064)
    assert np.array_equal(u1, u2[1000:]) and np.array_equal(v1, v2[1000:])
    u3, _ = O.rmat_raw(14, 0.57, 0.19, 0.19, 6, 1000, 64)
    assert not np.array_equal(u1, u3)


def _brute_csr(scale, ef, a, b, c, g):
    n = 1 << scale
    u, v = O.rmat_raw(scale, a, b, c, g, 0, ef << scale)
    rows = [set() for _ in range(n)]
    for x, y in zip(u.tolist(), v.tolist()):
        if x != y:
            rows[x].add(y)
            rows[y].add(x)
    return rows


@pytest.mark.parametrize("scale,abc,weighted", [(8, (0.57, 0.19, 0.19), False),
                                                (9, (0.65, 0.15, 0.15), True),
                                                (10, (0.25, 0.25, 0.25), False)])
def test_csr_equals_set_construction(scale, abc, weighted):
    g = O.rmat_csr(scale, 16, *abc, 11, weighted=weighted, nthreads=4)
    rows = _brute_csr(scale, 16, *abc, 11)
    assert g.n == 1 << scale
    for x in range(g.n):
        r = g.row(x).tolist()
        assert r == sorted(rows[x])
        if weighted:
            w = g.wt[int(g.off[x]):int(g.off[x + 1])].tolist()
            assert w == [O.pair_weight(11, x, y) for y in r]


def test_csr_invariants_scale14():
    g = O.rmat_csr(14, 16, 0.57, 0.19, 0.19, 14, weighted=True, nthreads=4)
    off, adj, wt = g.off.astype(np.int64), g.adj.astype(np.int64), g.wt
    assert off[0] == 0 and off[-1] == len(adj)
    deg = np.diff(off)
    src = np.repeat(np.arange(g.n), deg)
    # strictly ascending rows, no loops, ids in range
    same_row = src[1:] == src[:-1]
    assert np.all(adj[1:][same_row] > adj[:-1][same_row])
    assert np.all(adj != src)
    assert adj.max() < g.n
    # symmetric with symmetric weights
    key_f = src * g.n + adj
    key_r = adj * g.n + src
    order_f = np.argsort(key_f)
    order_r = np.argsort(key_r)
    assert np.array_equal(key_f[order_f], key_r[order_r])
    assert np.array_equal(wt[order_f], wt[order_r])
    assert wt.min() >= 1 and wt.max() <= 1000
    # weights roughly uniform on 1..1000
    assert abs(wt.mean() - 500.5) < 10


def test_csr_thread_count_invariant():
    g1 = O.rmat_csr(12, 16, 0.65, 0.15, 0.15, 7, nthreads=1)
    g2 = O.rmat_csr(12, 16, 0.65, 0.15, 0.15, 7, nthreads=8)
    assert np.array_equal(g1.off, g2.off) and np.array_equal(g1.adj, g2.adj)
