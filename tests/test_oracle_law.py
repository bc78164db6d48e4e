"""The oracle's draws follow node2vec's exact law (CPU only).

The reference law is computed by exact enumeration (oracle/brute.py) from the
model of Section 2.1 with real 1/p and 1/q and breadth-first distances, i.e.
independently of the integer multipliers, the membership test and both
sampling rules that the oracle uses.  Closed forms on special graphs pin the
enumerator itself.
"""
import itertools
import random
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle import brute

PQ = [0.25, 0.5, 1.0, 2.0, 4.0]
ALL_PQ = list(itertools.product(PQ, PQ))
RULES = [  # (d_rule, a_cap)
    (1024, 1024),          # default: rejection below the threshold
    (0, 1024),             # inverse CDF everywhere
    (0xFFFFFFFF, 1024),    # rejection everywhere
    (0xFFFFFFFF, 1),       # rejection with one attempt, fallback exercised
    (0xFFFFFFFF, 2),
]


def random_graph(n, p_edge, seed, weighted):
    rng = random.Random(seed)
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p_edge]
    weights = {e: rng.randint(1, 20) for e in edges} if weighted else None
    return O.CSR.from_edges(n, edges, weights)


def chi2_ok(obs, probs, thresh=1e-6):
    obs = np.asarray(obs, dtype=np.float64)
    probs = np.asarray(probs, dtype=np.float64)
    n = obs.sum()
    if len(obs) == 1:
        return obs[0] == n and probs[0] == 1.0
    exp = probs * n
    # every probability is strictly positive in these laws
    assert np.all(exp > 5)
    return stats.chisquare(obs, exp).pvalue > thresh


def law_vector(g, t, v, p, q, first):
    law = brute.transition_law(g.off, g.adj, g.wt, t, v, p, q, first=first)
    return [float(law[int(x)]) for x in g.row(v)]


def states(g):
    out = []
    for v in range(g.n):
        for t in g.row(v).tolist():
            out.append((t, v))
    return out


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("rule", RULES)
def test_single_move_law_random_graphs(weighted, rule):
    d_rule, a_cap = rule
    g = random_graph(7, 0.55, 17 + weighted, weighted)
    sts = states(g)
    rng = random.Random(3)
    for i, (t, v) in enumerate(rng.sample(sts, min(6, len(sts)))):
        p, q = ALL_PQ[(7 * i + 3 * weighted) % 25]
        for s in (0, 1):
            h = O.step_hist(g, t, v, s, 60_000, p, q, seed=1000 + i, d_rule=d_rule, a_cap=a_cap)
            assert chi2_ok(h, law_vector(g, t, v, p, q, first=(s == 0))), (t, v, s, p, q, h)


@pytest.mark.parametrize("p,q", ALL_PQ)
def test_single_move_law_all_pq(p, q):
    g = random_graph(8, 0.5, 5, False)
    for t, v in [(0, x) for x in g.row(0).tolist()][:2] + [(x, 0) for x in g.row(0).tolist()][:2]:
        h = O.step_hist(g, t, v, 3, 40_000, p, q, seed=77)
        assert chi2_ok(h, law_vector(g, t, v, p, q, False)), (t, v, p, q, h)


def test_brute_law_uses_distance_classes():
    # path 0-1-2-3 plus chord 0-2: from (0 -> 2) the neighbours of 2 are 0 (back),
    # 1 (common neighbour of 0 and 2) and 3 (distance 2)
    g = O.CSR.from_edges(4, [(0, 1), (1, 2), (2, 3), (0, 2)])
    law = brute.transition_law(g.off, g.adj, None, 0, 2, 0.5, 2.0)
    z = 2 + 1 + Fraction(1, 2)
    assert law == {0: 2 / z, 1: 1 / z, 3: Fraction(1, 2) / z}


def _closed_form_cases():
    cases = []
    for p, q in [(0.25, 4.0), (0.5, 2.0), (1.0, 0.5), (2.0, 0.25), (4.0, 1.0)]:
        P, Q = Fraction(p), Fraction(q)
        n = 6
        cyc = O.CSR.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
        cases.append(("cycle", cyc, 0, 1, 0, Q / (P + Q), p, q))
        n = 5
        kn = O.CSR.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
        cases.append(("clique", kn, 0, 1, 0, (1 / P) / (1 / P + n - 2), p, q))
        a, b = 3, 4  # vertices 0..2 on side A, 3..6 on side B
        kab = O.CSR.from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])
        cases.append(("bipartite", kab, 0, 3, 0, (1 / P) / (1 / P + (a - 1) / Q), p, q))
        k = 7  # centre 0, leaves 1..7
        star = O.CSR.from_edges(k + 1, [(0, i) for i in range(1, k + 1)])
        cases.append(("star-in", star, 1, 0, 1, (1 / P) / (1 / P + (k - 1) / Q), p, q))
        cases.append(("star-out", star, 0, 1, 0, Fraction(1), p, q))
    return cases


@pytest.mark.parametrize("case", _closed_form_cases(), ids=lambda c: f"{c[0]}-{c[6]}-{c[7]}")
def test_closed_forms(case):
    name, g, t, v, back, want, p, q = case
    # the enumerator agrees with the hand-derived closed form
    law = brute.transition_law(g.off, g.adj, None, t, v, p, q)
    assert law[back] == want
    # and the oracle's draws agree with it (binomial test)
    row = g.row(v).tolist()
    idx = row.index(back)
    N = 100_000
    for d_rule in (1024, 0):
        h = O.step_hist(g, t, v, 2, N, p, q, seed=9, d_rule=d_rule)
        k = int(h[idx])
        pw = float(want)
        if pw == 1.0:
            assert k == N
        else:
            assert stats.binomtest(k, N, pw).pvalue > 1e-6, (name, k, N, pw)


@pytest.mark.parametrize("weighted", [False, True])
def test_three_move_path_law(weighted):
    g = random_graph(6, 0.6, 41, weighted)
    p, q = 0.5, 2.0
    start = 0
    while int(g.off[start + 1] - g.off[start]) == 0:
        start += 1
    N = 200_000
    r = O.walk(g, np.full(N, start, dtype=np.uint32), 3, p, q, seed=12)
    law = brute.path_law(g.off, g.adj, g.wt, start, 3, p, q)
    keys = list(law.keys())
    index = {k: i for i, k in enumerate(keys)}
    obs = np.zeros(len(keys))
    for row in r["out"]:
        obs[index[tuple(int(x) for x in row)]] += 1
    probs = np.array([float(law[k]) for k in keys])
    big = probs * N > 5
    obs2 = np.append(obs[big], obs[~big].sum())
    pr2 = np.append(probs[big], probs[~big].sum())
    if pr2[-1] == 0:
        obs2, pr2 = obs2[:-1], pr2[:-1]
    assert stats.chisquare(obs2, pr2 * N).pvalue > 1e-6


@pytest.mark.parametrize("p,q", ALL_PQ)
def test_first_move_independent_of_rule_unweighted(p, q):
    # unweighted first move: rejection accepts attempt 0 at j = hi64(R1, d) and the
    # inverse CDF picks floor of hi64(R1, d): the two rules give the same vertex
    g = O.rmat_csr(10, 16, 0.57, 0.19, 0.19, 10)
    starts = np.arange(g.n, dtype=np.uint32)
    a = O.walk(g, starts, 1, p, q, seed=5, d_rule=1024)["out"]
    b = O.walk(g, starts, 1, p, q, seed=5, d_rule=0)["out"]
    c = O.walk(g, starts, 1, p, q, seed=5, d_rule=0xFFFFFFFF)["out"]
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_unbiased_walk_identical_for_every_rule():
    # p = q = 1, unweighted: all multipliers are 4, rejection accepts attempt 0 at
    # j = hi64(R1, d) and the inverse CDF picks floor(hi64(R1, 4d) / 4) = hi64(R1, d)
    g = O.rmat_csr(11, 16, 0.57, 0.19, 0.19, 21)
    starts = np.arange(g.n, dtype=np.uint32)
    outs = [O.walk(g, starts, 20, 1.0, 1.0, seed=8, d_rule=d)["out"] for d in (0, 7, 1024, 0xFFFFFFFF)]
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_first_order_stationary_distribution():
    # p = q = 1 is a first-order walk; on a connected non-bipartite graph its visit
    # frequencies converge to weighted degree / total weight
    g = random_graph(9, 0.5, 8, True)
    deg = g.degree()
    assert np.all(deg > 0)
    strength = np.array([int(g.wt[int(g.off[v]):int(g.off[v + 1])].sum()) for v in range(g.n)], float)
    W = 400
    L = 2000
    r = O.walk(g, np.arange(W, dtype=np.uint32) % g.n, L, 1.0, 1.0, seed=4, want_counts=True)
    freq = r["cnt"] / r["cnt"].sum()
    pi = strength / strength.sum()
    assert np.abs(freq - pi).sum() < 0.02, (freq, pi)
