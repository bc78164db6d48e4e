"""Pins of the oracle's algorithmic-bytes models and of its checksum hash (CPU).

Every expected figure below is derived by hand in the comment beside it, from
the layout of the arrays: byte b of an array lies in 64-byte line b // 64,
off is u64 (off[v] at byte 8v), adj u32 (entry e at byte 4e), wt and wmax
u16.  The isolated model charges the distinct lines one move must read plus 4
bytes of output; where the charge depends on the move's draw, the draw is
taken from the pure-Python Philox (written separately from the C one) and
the rule's integer arithmetic, and the table of hand-derived costs is
indexed by it.
"""
import numpy as np

import oracle as O
from oracle.philox_ref import philox4x32

SEED = 0x1234_5678_9ABC


def k8(weight=None):
    edges = [(a, b) for a in range(8) for b in range(a + 1, 8)]
    wts = None if weight is None else {(a, b): weight for a, b in edges}
    return O.CSR.from_edges(8, edges, wts)


def star(leaves):
    return O.CSR.from_edges(leaves + 1, [(0, k) for k in range(1, leaves + 1)])


def draw(wid, s, k):
    r = philox4x32((SEED & 0xFFFFFFFF, SEED >> 32), (wid, s, k, 0))
    return (r[0] << 32) | r[1], (r[2] << 32) | r[3]


def hi64(x, y):
    return (x * y) >> 64


# K8 layout: off[v] at byte 8v, so off[0..7] share line 0 and off[8] is in line 1.
# Row v holds the 7 other vertices at entries 7v .. 7v+6: row 3 = entries 21..27
# (line 1), row 4 = 28..34 (lines 1 and 2), row 7 = 49..55 (line 3).

def test_first_move_unweighted():
    g = k8()
    for wid in range(40):
        # v = 7: off[7] (line 0) and off[8] (line 1), the accepted entry (line 3): 3 lines
        b, _ = O.step_cost(g, SEED, wid, 0, O.SENT, 7, 1.0, 1.0)
        assert b == 3 * 64 + 4
        # v = 0: off[0], off[1] in line 0, the entry in line 0 of adj: 2 lines
        b, _ = O.step_cost(g, SEED, wid, 0, O.SENT, 0, 1.0, 1.0)
        assert b == 2 * 64 + 4


def test_first_move_weighted():
    g = k8(weight=7)
    for wid in range(40):
        # E = wmax = 7, u < 7 = w: attempt 0 accepts.  off lines 0 and 1, wmax[7] (byte 14,
        # line 0 of wmax), wt of entry 49+j (bytes 98..110, line 1 of wt), the entry (line 3)
        b, _ = O.step_cost(g, SEED, wid, 0, O.SENT, 7, 1.0, 1.0)
        assert b == 5 * 64 + 4


def test_accept_without_search():
    # p = q = 1: every multiplier is 4 = A_max, so attempt 0 accepts with no membership test.
    # t = 3 sits at index 3 of N(7): drawing it needs no read (2 off lines); any other index
    # reads its entry (line 3)
    g = k8()
    seen = set()
    for wid in range(200):
        R1, _ = draw(wid, 1, 0)
        j = hi64(R1, 7)
        want = (2 if j == 3 else 3) * 64 + 4
        b, x = O.step_cost(g, SEED, wid, 1, 3, 7, 1.0, 1.0)
        assert b == want and x == j
        seen.add(j == 3)
    assert seen == {True, False}


def test_accept_after_search():
    # p = 1, q = 4: A = (4, 4, 1), E = 4.  At v = 7 after t = 4 (index 4 of N(7)):
    #   j = 4          -> t itself, no read                                  2 lines
    #   j != 4, u = 0  -> u < A_out * 1 accepts without the test              3 lines
    #   j != 4, u >= 1 -> x = j is searched in N(4) = [0,1,2,3,5,6,7] at entries 28..34:
    #                     x <= 3 probes entries 31, 29, 28 / 30 (line 1)      4 lines
    #                     x in {5, 6} probes 31 (line 1), 33 and 32 (line 2)  5 lines
    # every x != t is a neighbour of t, so attempt 0 always accepts
    g = k8()
    cases = set()
    for wid in range(400):
        R1, R2 = draw(wid, 1, 0)
        j, u = hi64(R1, 7), hi64(R2, 4)
        if j == 4:
            lines, case = 2, "t"
        elif u == 0:
            lines, case = 3, "free"
        elif j <= 3:
            lines, case = 4, "search-low"
        else:
            lines, case = 5, "search-high"
        b, x = O.step_cost(g, SEED, wid, 1, 4, 7, 1.0, 4.0)
        assert b == lines * 64 + 4, (wid, j, u)
        assert x == j
        cases.add(case)
    assert cases == {"t", "free", "search-low", "search-high"}


def test_cap_fallback_to_inverse_cdf():
    # p = 4, q = 1: A = (1, 4, 4), E = 4, a_cap = 1.  At v = 7 after t = 4:
    #   j != 4          -> u < 4 accepts without the test                      3 lines
    #   j = 4, u = 0    -> accepts (u < A_ret)                                 2 lines
    #   j = 4, u >= 1   -> rejected; inverse CDF.  Merge: off (2) + N(7) (line 3) + N(4)
    #                      (lines 1, 2) = 5.  Search: off (2) + N(4) (lines 1, 2) + every
    #                      search in N(7) (line 3) = 5.  The cheaper: 5 lines
    g = k8()
    cases = set()
    for wid in range(400):
        R1, R2 = draw(wid, 1, 0)
        j, u = hi64(R1, 7), hi64(R2, 4)
        lines = 3 if j != 4 else (2 if u == 0 else 5)
        b, _ = O.step_cost(g, SEED, wid, 1, 4, 7, 4.0, 1.0, a_cap=1)
        assert b == lines * 64 + 4, (wid, j, u)
        cases.add(lines)
    assert cases == {2, 3, 5}


def test_dense_hub():
    # d_rule = 6 makes every K8 vertex a hub.  v = 7 after t = 4: merge 5 lines, search 5
    # lines (as in the fallback); first move at v = 7: off (2) + the chosen entry (line 3)
    g = k8()
    for wid in range(20):
        b, _ = O.step_cost(g, SEED, wid, 1, 4, 7, 0.5, 2.0, d_rule=6)
        assert b == 5 * 64 + 4
        b, _ = O.step_cost(g, SEED, wid, 0, O.SENT, 7, 0.5, 2.0, d_rule=6)
        assert b == 3 * 64 + 4


def star_draw(wid, A_ret, A_out):
    # inverse CDF at the centre of star(200) after leaf 5 (index 4): pi = A_ret there,
    # A_out elsewhere (no leaf neighbours leaf 5)
    R1, _ = draw(wid, 1, 0)
    S = A_ret + 199 * A_out
    r = hi64(R1, S)
    P = 0
    for i in range(200):
        P += A_ret if i == 4 else A_out
        if P > r:
            return i


def test_sparse_hub():
    # star(200), d_rule 10: the centre's row is entries 0..199 (lines 0..12), leaf k's row
    # is entry 199+k (leaf 5: entry 204, line 12); off[0], off[1] in line 0.
    # At the centre after leaf 5: merge = 1 + 13 = 14 lines.  Search: N(5) (line 12), the
    # search of 0 in the centre's row probes entries 100, 50, 25, 12, 6, 3, 1, 0 (lines 6,
    # 3, 1, 0), plus the chosen entry's line j // 16: 1 + 5 lines, or 1 + 6 when j // 16 is
    # none of 0, 1, 3, 6, 12
    g = star(200)
    seen = set()
    for wid in range(300):
        j = star_draw(wid, 8, 2)
        lines = 6 if j // 16 in (0, 1, 3, 6, 12) else 7
        b, x = O.step_cost(g, SEED, wid, 1, 5, 0, 0.5, 2.0, d_rule=10)
        assert x == j + 1 and b == lines * 64 + 4, (wid, j)
        seen.add(lines)
    assert seen == {6, 7}


def test_fn_approx_move():
    # FN-Approx at the star's centre after leaf 5 (d_t = 1 <= d_rule < 200): at p = q = 1 the
    # bounds coincide, so the move is drawn from the static weights: off (line 0) and the
    # chosen entry j = hi64(R1, 200): 2 lines.  The exact rule pays the search (6 or 7)
    g = star(200)
    for wid in range(100):
        R1, _ = draw(wid, 1, 0)
        j = hi64(R1, 200)
        b, x = O.step_cost(g, SEED, wid, 1, 5, 0, 1.0, 1.0, d_rule=10, approx_t=1000)
        assert x == j + 1 and b == 2 * 64 + 4
        b_exact, _ = O.step_cost(g, SEED, wid, 1, 5, 0, 1.0, 1.0, d_rule=10)
        assert b_exact in (6 * 64 + 4, 7 * 64 + 4)


# ---------------------------------------------------------------- memo-aware model

def test_memo_closed_forms_by_hand():
    assert [O.memo_off_lines(v) for v in (0, 6, 7, 8)] == [1, 1, 2, 1]  # bytes 8v .. 8v+15
    assert [O.memo_search_levels(d) for d in (1, 32, 33, 64, 65, 200, 1000)] == [1, 1, 2, 2, 3, 4, 6]
    g = star(200)
    # centre (13 lines) with leaf 5 (1 line): merge 14, search 1 + 1 x levels(200) = 5
    assert O.memo_pair_lines(g.off, 0, 5) == 5 == O.memo_pair_lines(g.off, 5, 0)
    assert O.memo_cold_lines(g.off, 5, 0) == 5
    # weighted: both add the centre's weights, bytes 0..399 of wt (7 lines)
    assert O.memo_cold_lines(g.off, 5, 0, weighted=True) == 12
    # at leaf 5 after the centre: merge 1 + 13 = 14, search 13 + 200 x 1 = 213
    assert O.memo_cold_lines(g.off, 0, 5) == 14
    # warm at degree 100000 after degree 3000: 196 tiles, segments of 4 x 512 (49, a row of 50
    # x 6 = 300 bytes: 5 lines), half 1024 entries (64 lines), ceil(3000 x 1024 / 100000) = 31
    # entries of N(t) (2 lines)
    off = np.array([0, 100000, 103000], dtype=np.uint64)
    assert O.memo_warm_lines(off, 1, 0) == 71
    # degree 600 after 100: two segments of 512 (a 12-byte row: 1 line), half 256 entries (16
    # lines), 43 entries (3 lines)
    off = np.array([0, 600, 700], dtype=np.uint64)
    assert O.memo_warm_lines(off, 1, 0) == 20


def test_memo_row_bytes_by_hand():
    # 6 bytes per segment (22 weighted), segments of whole 512-entry tiles, at most 64 of them,
    # rounded up to an even count
    assert [O.memo_row_bytes(d) for d in (1, 512, 1025, 3000, 32768)] == [12, 12, 24, 36, 384]
    # 65 tiles: two per segment, 33 segments, 34 in the row; 196 tiles: four per segment, 49
    assert O.memo_row_bytes(32769) == 6 * 34 and O.memo_row_bytes(100000) == 6 * 50
    assert O.memo_row_bytes(127 * 512 * 64) == 384 and O.memo_row_bytes(127 * 512 * 64, True) == 1408
    assert O.memo_row_bytes(600, True) == 44 and O.memo_row_bytes(100000, True) == 22 * 50


def test_memo_pass_bytes_by_hand():
    S = O.SENT
    g = star(200)
    out = np.array([[5, 0, 7, 0, 5], [9, 0, 5, S, S], [7, 0, 7, 0, 7]], dtype=np.uint32)
    # hub moves (at the centre, s >= 1): row 0 s = 1, 3; row 1 s = 1; row 2 s = 1, 3 -> 5.
    # other moves: row 0 s = 0, 2; row 1 s = 0; row 2 s = 0, 2 -> 5.
    # At the centre after a leaf the summary would cost 15 lines (row 1, half segment of 200
    # entries 13, one entry of N(t) 1) against 5 lines for searching the leaf's one
    # neighbour: every move takes the search (5 lines + off 1) and no intersection is kept
    cold = dict(hub_bytes=5 * (6 * 64 + 4), hub_moves=5, other_moves=5, intersections=0, warm_moves=0)
    assert O.memo_pass_bytes(g.off, out, 4, d_rule=10) == cold
    assert O.memo_pass_bytes(g.off, out, 4, d_rule=10, memo=False) == cold


def test_memo_pass_bytes_with_summaries_by_hand():
    # rows of degree 100000 (vertex 0: entries 0..99999, lines 0..6249), 3000 (vertex 1:
    # entries 100000..102999, lines 6250..6437) and 1 (vertex 2: entry 103000, line 6437);
    # off lines: 1 each.  d_rule 10.  The model reads offsets only.
    off = np.array([0, 100000, 103000, 103001], dtype=np.uint64)
    out = np.array([[2, 0, 1, 0, 1, 0]], dtype=np.uint32)
    # s = 0 at vertex 2: another move.
    # s = 1 at 0 after 2: summary 5 + 64 + 1 = 70 lines, search 1 + 1 x 13 = 14: 14 lines
    # s = 2 at 1 after 0: summary 1 (six segments: 36 bytes) + 16 (half of a 512 segment) +
    #   534 (8534 entries of N(0)) = 551 lines, cold min(6250 + 188, 6250 + 100000 x 8) = 6438:
    #   551; key {0, 1}
    # s = 3 at 0 after 1: summary 71 (as in the closed forms), cold 6438: 71; key {0, 1}
    # s = 4 at 1 after 0: 551; key {0, 1}
    # one intersection {0, 1}: merge 6250 + 188 = 6438, search 188 + 3000 x 13 = 39188
    hub = (1 + 14) * 64 + 4 + (1 + 551) * 64 + 4 + (1 + 71) * 64 + 4 + (1 + 551) * 64 + 4 + 6438 * 64
    r = O.memo_pass_bytes(off, out, 5, d_rule=10)
    assert r == dict(hub_bytes=hub, hub_moves=4, other_moves=1, intersections=1, warm_moves=3)
    # no summaries: 14, then 6438 for each of the others
    r = O.memo_pass_bytes(off, out, 5, d_rule=10, memo=False)
    assert r == dict(hub_bytes=(1 + 14) * 64 + 4 + 3 * ((1 + 6438) * 64 + 4), hub_moves=4, other_moves=1,
                     intersections=0, warm_moves=0)
    # vertex 1 keeps no summary (threshold 3001): its moves pay 6438, and the summary of
    # vertex 0 serves the directed key (0, 1) only
    r = O.memo_pass_bytes(off, out, 5, d_rule=10, memo_min=3001)
    assert r == dict(hub_bytes=(1 + 14) * 64 + 4 + 2 * ((1 + 6438) * 64 + 4) + (1 + 71) * 64 + 4 + 6438 * 64,
                     hub_moves=4, other_moves=1, intersections=1, warm_moves=1)


def test_memo_pass_bytes_weighted_by_hand():
    # the same rows, weighted: a summary row holds four 32-bit sums per segment beside the counts
    # and hints (22 bytes per segment: 1100 bytes, 18 lines, for the 50 of vertex 0; 132 bytes,
    # 3 lines, for the 6 of vertex 1), the half segment's weights are read too, every key is
    # directed (v, t), and building a summary costs the directed cold evaluation, weights of
    # N(v) included (vertex 0: 100000 weights, 3125 lines; vertex 1: bytes 200000..205999 of
    # wt, 94 lines).
    off = np.array([0, 100000, 103000, 103001], dtype=np.uint64)
    out = np.array([[2, 0, 1, 0, 1, 0]], dtype=np.uint32)
    assert O.memo_warm_lines(off, 1, 0, weighted=True) == 18 + 64 + 32 + 2
    # s = 1 at 0 after 2: summary 18 + 64 + 32 + 1 = 115 against cold min(6250 + 1, 1 + 13) + 3125
    #   = 3139: 115, key (0, 2)
    # s = 2 at 1 after 0: 3 + 16 + 8 + 534 = 561 against min(188 + 6250, 6250 + 800000) + 94
    #   = 6532: 561, key (1, 0); s = 4 the same key again
    # s = 3 at 0 after 1: 116 against min(6250 + 188, 188 + 39000) + 3125 = 9563: 116, key (0, 1)
    hub = ((1 + 115) + (1 + 561) + (1 + 116) + (1 + 561)) * 64 + 4 * 4 + (3139 + 6532 + 9563) * 64
    r = O.memo_pass_bytes(off, out, 5, d_rule=10, weighted=True)
    assert r == dict(hub_bytes=hub, hub_moves=4, other_moves=1, intersections=3, warm_moves=4)


def test_memo_model_is_below_the_isolated_model_on_repeated_pairs():
    # on a skewed R-MAT graph with four walks per vertex, hub pairs repeat: the memo-aware
    # bytes of the pass stay well below the isolated bytes of the same moves, and without
    # summaries the closed forms sit near the isolated line counts
    g = O.rmat_csr(14, 16, 0.65, 0.15, 0.15, 14)
    starts = np.tile(np.arange(g.n, dtype=np.uint32), 4)
    wids = np.arange(len(starts), dtype=np.uint64)
    out = O.walk(g, starts, 20, 0.25, 4.0, 3, wids=wids)["out"]
    cls = O.walk_cost_classes(g, starts, wids, 20, 0.25, 4.0, 3)
    memo = O.memo_pass_bytes(g.off, out, 20)
    none = O.memo_pass_bytes(g.off, out, 20, memo=False)
    assert memo["hub_moves"] == cls[1] and memo["other_moves"] == cls[3]
    assert memo["intersections"] < memo["warm_moves"] / 2
    assert memo["hub_bytes"] < 0.8 * cls[0]
    assert 0.8 * cls[0] < none["hub_bytes"] < 1.5 * cls[0]


# ---------------------------------------------------------------- checksum hash

def test_entry_hash_against_the_python_philox():
    # H(w, c, x) = r0 * 2^32 + r1 of Philox(key = seed; ctr = (w, c, x, 3))
    rng = np.random.default_rng(5)
    for _ in range(2000):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        w, c, x = (int(v) for v in rng.integers(0, 2**32, size=3, dtype=np.uint64))
        r = philox4x32((seed & 0xFFFFFFFF, seed >> 32), (w, c, x, 3))
        assert O.entry_hash(seed, w, c, x) == (r[0] << 32) | r[1]


def test_checksum_of_a_walk_by_hand():
    # the oracle's checksum of a walk equals the sum of the Python hashes of its entries
    g = k8()
    starts = np.array([1, 6], dtype=np.uint32)
    r = O.walk(g, starts, 5, 0.5, 2.0, SEED, walk_base=77)
    total = 0
    for i, row in enumerate(r["out"]):
        for c, x in enumerate(row):
            h = philox4x32((SEED & 0xFFFFFFFF, SEED >> 32), (77 + i, c, int(x), 3))
            total = (total + ((h[0] << 32) | h[1])) & 0xFFFFFFFFFFFFFFFF
    assert r["checksum"] == total
