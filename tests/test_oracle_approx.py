"""Pins of the oracle's FN-Approx rule (Section 3.4, Eqs. 2 and 3).

The bounds are checked against the exact transition law of the paper's model
(rational arithmetic, distances by breadth-first search) on small graphs: they
must hold for every move, and on the graphs that realise the extreme cases
they must be attained, so a dropped term, a swapped multiplier or a wrong
count of common neighbours fails.  The approximate draw is checked against
the static-weight law, and approximate walks against exact walks."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle import brute

PQ = [0.25, 0.5, 1.0, 2.0, 4.0]


def _csr(n, edges, weights=None):
    """Symmetric CSR from undirected edges (optional weight per edge)."""
    rows = [dict() for _ in range(n)]
    for k, (a, b) in enumerate(edges):
        w = 1 if weights is None else int(weights[k])
        rows[a][b] = w
        rows[b][a] = w
    off = np.zeros(n + 1, dtype=np.uint64)
    adj, wt = [], []
    for v in range(n):
        for x in sorted(rows[v]):
            adj.append(x)
            wt.append(rows[v][x])
        off[v + 1] = len(adj)
    return O.CSR(off, np.array(adj, dtype=np.uint32), None if weights is None else np.array(wt, dtype=np.uint16))


def _random_graph(rng, n, m, weighted):
    edges = set()
    while len(edges) < m:
        a, b = rng.integers(0, n, size=2)
        if a != b:
            edges.add((int(min(a, b)), int(max(a, b))))
    edges = sorted(edges)
    w = rng.integers(1, 9, size=len(edges)) if weighted else None
    return _csr(n, edges, w)


def _deg(g, v):
    return int(g.off[v + 1] - g.off[v])


@pytest.mark.parametrize("weighted", [False, True])
def test_bounds_hold_for_every_move(weighted):
    rng = np.random.default_rng(5 + weighted)
    for trial in range(6):
        g = _random_graph(rng, 14, 40, weighted)
        wlo = int(g.wt.min()) if weighted else 1
        whi = int(g.wt.max()) if weighted else 1
        for p, q in itertools.product(PQ, PQ):
            for u in range(g.n):
                for v in g.adj[int(g.off[u]):int(g.off[u + 1])]:
                    v = int(v)
                    lb, ub = O.approx_bounds(_deg(g, u), _deg(g, v), p, q, wlo, whi)
                    law = brute.transition_law(g.off, g.adj, g.wt, u, v, p, q)
                    for x, pr in law.items():
                        if x != u:
                            assert lb <= pr <= ub, (trial, p, q, u, v, x, pr, lb, ub)


def _fan(k, m):
    """v = 0, u = 1, commons 2..k+1 (adjacent to u and v), others k+2..k+m+1
    (adjacent to v only): d_u = k + 1, d_v = 1 + k + m."""
    edges = [(0, 1)] + [(0, 2 + i) for i in range(k)] + [(1, 2 + i) for i in range(k)]
    edges += [(0, 2 + k + i) for i in range(m)]
    return _csr(2 + k + m, edges)


@pytest.mark.parametrize("k,m", [(0, 5), (3, 4), (6, 1), (2, 9)])
def test_bounds_attained_on_extreme_graphs(k, m):
    # an outer neighbour x of v with all d_u - 1 other neighbours of u common:
    # its probability is the largest possible when 1/q >= 1 and the smallest
    # possible when 1/q <= 1
    g = _fan(k, m)
    x = 2 + k
    for p, q in itertools.product(PQ, PQ):
        law = brute.transition_law(g.off, g.adj, None, 1, 0, p, q)
        lb, ub = O.approx_bounds(k + 1, 1 + k + m, p, q)
        if q <= 1:
            assert law[x] == ub, (p, q)
        if q >= 1:
            assert law[x] == lb, (p, q)
        if q == 1:
            assert lb == ub


def test_paper_case_matches_eq2():
    # Eq. 2 (1/p <= 1 <= 1/q): LB = Wmin / ((1/p + (d_v - 1)/q) Wmax)
    for p, q in [(1.0, 1.0), (2.0, 0.5), (4.0, 0.25), (1.0, 0.5), (2.0, 1.0)]:
        for du, dv, wlo, whi in [(3, 5000, 1, 1), (10, 20000, 1, 1), (5, 1500, 2, 7)]:
            lb, _ = O.approx_bounds(du, dv, p, q, wlo, whi)
            ip, iq = 1 / Fraction(p), 1 / Fraction(q)
            assert lb == Fraction(wlo) / ((ip + (dv - 1) * iq) * whi)


def test_paper_case_matches_eq3_with_reachable_common_neighbours():
    # Eq. 3 (1/p <= 1 <= 1/q): UB = (Wmax/q) / ((1/p + d_u + (d_v - d_u - 1)/q) Wmin)
    # assumes d_u common neighbours; at most d_u - 1 are possible (u's
    # neighbour v is not a neighbour of v), and with d_u - 1 in place of d_u
    # the oracle's bound is Eq. 3 exactly, and never above Eq. 3 as printed
    for p, q in [(1.0, 0.5), (2.0, 0.5), (4.0, 0.25), (1.0, 1.0), (2.0, 1.0)]:
        for du, dv, wlo, whi in [(3, 5000, 1, 1), (10, 20000, 1, 1), (5, 1500, 2, 7), (1, 1025, 1, 1)]:
            _, ub = O.approx_bounds(du, dv, p, q, wlo, whi)
            ip, iq = 1 / Fraction(p), 1 / Fraction(q)

            def eq3(c):
                return (whi * iq) / ((ip + c + (dv - c - 1) * iq) * wlo)

            assert ub == eq3(du - 1)
            assert ub <= eq3(du)


def test_gap_decision_is_exact_at_extreme_sizes():
    rng = np.random.default_rng(3)
    cases = [(1, 2), (1, 2**32 - 1), (1024, 2**32 - 1), (2**31, 2**32 - 1), (7, 1025), (1024, 1025)]
    cases += [(int(a), int(b)) for a, b in zip(rng.integers(1, 1025, 60), rng.integers(1025, 2**32, 60))]
    for du, dv in cases:
        for p, q in [(0.25, 4.0), (4.0, 0.25), (0.5, 2.0), (2.0, 0.5), (1.0, 1.0)]:
            for wlo, whi in [(1, 1), (1, 65535), (65535, 65535), (3, 1000)]:
                lb, ub = O.approx_bounds(du, dv, p, q, wlo, whi)
                for T in (1, 1000, 123457, 2**32 - 1):
                    assert O.approx_gap_below(du, dv, p, q, T, wlo, whi) == (ub - lb < Fraction(1, T))


def _hub_graph():
    """A hub v = 0 of degree 40 with a spoke u = 1 of degree 3 (two commons)."""
    edges = [(0, i) for i in range(1, 41)] + [(1, 2), (1, 3)] + [(5, 6), (7, 8), (8, 9)]
    return _csr(41, edges)


def test_approx_move_follows_the_static_weights():
    g = _hub_graph()
    d_rule = 8
    p, q = 0.5, 2.0
    lb, ub = O.approx_bounds(3, 40, p, q)
    T = int(1 / (ub - lb))  # threshold 1/T just above the gap: the move is approximated
    assert O.approx_applies(g, 1, 0, p, q, T, d_rule=d_rule)
    assert not O.approx_applies(g, 1, 0, p, q, T + 1, d_rule=d_rule)
    assert not O.approx_applies(g, 1, 0, p, q, T, d_rule=40)  # v not popular
    assert not O.approx_applies(g, 1, 0, p, q, T, d_rule=2)   # u popular too
    draws = 200000
    h_apx = O.step_hist(g, 1, 0, 1, draws, p, q, seed=9, d_rule=d_rule, approx_t=T).astype(float)
    h_ex = O.step_hist(g, 1, 0, 1, draws, p, q, seed=9, d_rule=d_rule).astype(float)
    nb = [int(x) for x in g.adj[int(g.off[0]):int(g.off[1])]]
    first = brute.transition_law(g.off, g.adj, None, 1, 0, p, q, first=True)
    second = brute.transition_law(g.off, g.adj, None, 1, 0, p, q)

    def chi2(h, law):
        e = np.array([float(law[x]) for x in nb]) * draws
        return float(((h - e) ** 2 / e).sum())

    # 39 degrees of freedom: the 0.9999 quantile is about 80
    assert chi2(h_apx, first) < 80 and chi2(h_ex, second) < 80
    assert chi2(h_apx, second) > 400 and chi2(h_ex, first) > 400


def test_approx_walks_differ_only_at_approximated_moves():
    og = O.rmat_csr(11, 16, 0.57, 0.19, 0.19, 11, weighted=False, nthreads=8)
    n, L, d_rule = og.n, 20, 64
    starts = np.arange(n, dtype=np.uint32)
    for p, q in [(0.5, 2.0), (2.0, 0.5), (1.0, 1.0)]:
        ex = O.walk(og, starts, L, p, q, 4, d_rule=d_rule)["out"]
        ap = O.walk(og, starts, L, p, q, 4, d_rule=d_rule, approx_t=100)["out"]
        diff_rows = np.nonzero((ex != ap).any(axis=1))[0]
        if p == q == 1.0:
            # both laws are w / sum(w), and the exact rule's index
            # floor(hi64(R, 4 S) / 4) equals the first-order hi64(R, S)
            assert len(diff_rows) == 0
            continue
        assert len(diff_rows) > 0
        for i in diff_rows:
            c = int(np.nonzero(ex[i] != ap[i])[0][0])
            assert c >= 2  # the first move is first-order in both
            t, v = int(ex[i][c - 2]), int(ex[i][c - 1])
            assert O.approx_applies(og, t, v, p, q, 100, d_rule=d_rule)
        # every approximate move still follows an edge
        for row in ap[:200]:
            for a, b in zip(row[:-1], row[1:]):
                if b == O.SENT:
                    break
                nb = og.adj[int(og.off[a]):int(og.off[a + 1])]
                assert int(b) in set(int(x) for x in nb)
    # no popular vertex: nothing is approximated
    big = int(np.diff(og.off.astype(np.int64)).max())
    ex = O.walk(og, starts, L, 0.5, 2.0, 4, d_rule=big)["out"]
    ap = O.walk(og, starts, L, 0.5, 2.0, 4, d_rule=big, approx_t=1)["out"]
    assert np.array_equal(ex, ap)
    # threshold 0 is the exact rule
    assert np.array_equal(O.walk(og, starts, L, 0.5, 2.0, 4, d_rule=d_rule, approx_t=0)["out"],
                          O.walk(og, starts, L, 0.5, 2.0, 4, d_rule=d_rule)["out"])


def test_distance_report_measures_the_two_laws():
    from oracle.approx_distance import tv_distance
    g = _hub_graph()
    # p = q = 1: the exact law is the static-weight law
    assert tv_distance(g, 1, 0, 1.0, 1.0) == pytest.approx(0.0, abs=1e-15)
    # otherwise the distance equals half the L1 gap of the enumerated laws
    for p, q in [(0.5, 2.0), (2.0, 0.5), (4.0, 0.25)]:
        second = brute.transition_law(g.off, g.adj, None, 1, 0, p, q)
        first = brute.transition_law(g.off, g.adj, None, 1, 0, p, q, first=True)
        want = sum(abs(second[x] - first[x]) for x in second) / 2
        assert tv_distance(g, 1, 0, p, q) == pytest.approx(float(want), rel=1e-12)


def test_uniform_weights_walk_like_unweighted():
    # Scaling every weight by c changes no draw: floor(hi64(R, c S) / c) equals
    # hi64(R, S), rejection compares u < c pi as floor(u / c) < pi, and the
    # FN-Approx bounds are ratios of weights.  So a graph whose weights all
    # equal 7 walks exactly like the unweighted graph, exact rule or not.
    og = O.rmat_csr(10, 16, 0.65, 0.15, 0.15, 10, weighted=False, nthreads=8)
    w7 = O.CSR(og.off, og.adj, np.full(og.m, 7, dtype=np.uint16))
    starts = np.tile(np.arange(og.n, dtype=np.uint32), 3)
    for p, q in [(0.5, 2.0), (2.0, 0.5), (0.25, 4.0)]:
        for T in (0, 50):
            a = O.walk(og, starts, 20, p, q, 5, d_rule=64, approx_t=T)["out"]
            b = O.walk(w7, starts, 20, p, q, 5, d_rule=64, approx_t=T)["out"]
            assert np.array_equal(a, b), (p, q, T)
    exact = O.walk(og, starts, 20, 0.5, 2.0, 5, d_rule=64)["out"]
    assert not np.array_equal(exact, O.walk(og, starts, 20, 0.5, 2.0, 5, d_rule=64, approx_t=50)["out"])
