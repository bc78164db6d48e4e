"""Exact node2vec transition law by enumeration (test infrastructure only).

For a tiny graph this computes, with exact rationals, the probability of each
next vertex given the previous vertex t and the current vertex v, straight
from the model of Section 2.1: the weight of neighbour x of v is w_vx times
1/p when x == t, 1 when x is a neighbour of t, 1/q otherwise (distance 0, 1
or 2 from t), and the first move of a walk uses the edge weights alone
(Algorithm 1).  It uses real-valued 1/p and 1/q, not the integer multipliers
of the draw rule, so that it pins the rule to the paper's definition.  The
distance is computed by breadth-first search from t, not by a membership test.
"""
from __future__ import annotations

from collections import deque
from fractions import Fraction


def _neighbours(off, adj, v):
    return [int(x) for x in adj[int(off[v]):int(off[v + 1])]]


def _weights(off, wt, v):
    d = int(off[v + 1] - off[v])
    if wt is None:
        return [1] * d
    return [int(x) for x in wt[int(off[v]):int(off[v + 1])]]


def distances_from(off, adj, t):
    """Hop distances from t by breadth-first search."""
    n = len(off) - 1
    dist = [None] * n
    dist[t] = 0
    dq = deque([t])
    while dq:
        a = dq.popleft()
        for b in _neighbours(off, adj, a):
            if dist[b] is None:
                dist[b] = dist[a] + 1
                dq.append(b)
    return dist


def transition_law(off, adj, wt, t, v, p, q, first=False):
    """dict x -> Fraction, P(next = x | previous t, current v)."""
    p = Fraction(p).limit_denominator(1000)
    q = Fraction(q).limit_denominator(1000)
    nbrs = _neighbours(off, adj, v)
    ws = _weights(off, wt, v)
    if not nbrs:
        return {}
    if first:
        alphas = [Fraction(1)] * len(nbrs)
    else:
        dist = distances_from(off, adj, t)
        alphas = []
        for x in nbrs:
            dx = dist[x]
            if dx == 0:
                alphas.append(1 / p)
            elif dx == 1:
                alphas.append(Fraction(1))
            else:
                alphas.append(1 / q)
    un = [Fraction(w) * a for w, a in zip(ws, alphas)]
    tot = sum(un)
    return {x: u / tot for x, u in zip(nbrs, un)}


def path_law(off, adj, wt, start, steps, p, q):
    """Exact distribution of the first `steps` moves of a walk from `start`.

    Returns dict tuple(path including start) -> Fraction."""
    laws = {(start,): Fraction(1)}
    for s in range(steps):
        nxt = {}
        for path, pr in laws.items():
            v = path[-1]
            t = path[-2] if len(path) >= 2 else None
            law = transition_law(off, adj, wt, t if t is not None else v, v, p, q, first=(s == 0))
            if not law:
                nxt[path] = nxt.get(path, 0) + pr
                continue
            for x, px in law.items():
                key = path + (x,)
                nxt[key] = nxt.get(key, 0) + pr * px
        laws = nxt
    return laws
