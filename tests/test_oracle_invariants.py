"""Invariants of the oracle's walks, counts and checksum (CPU only)."""
import numpy as np
import pytest

import oracle as O

SENT = O.SENT


@pytest.fixture(scope="module")
def g12():
    return O.rmat_csr(12, 16, 0.57, 0.19, 0.19, 12)


@pytest.fixture(scope="module")
def g11w():
    return O.rmat_csr(11, 16, 0.65, 0.15, 0.15, 20, weighted=True)


def check_walks(g, starts, out, L):
    assert out.shape == (len(starts), L + 1)
    assert np.array_equal(out[:, 0], starts)
    for i, row in enumerate(out):
        ended = False
        for s in range(L):
            a, b = int(row[s]), int(row[s + 1])
            if ended or b == SENT:
                ended = True
                assert b == SENT
                continue
            r = g.row(a)
            assert len(r) > 0
            k = np.searchsorted(r, b)
            assert k < len(r) and r[k] == b, (i, s, a, b)
        if int(g.off[starts[i] + 1] - g.off[starts[i]]) == 0:
            assert np.all(row[1:] == SENT)


@pytest.mark.parametrize("pq", [(0.5, 2.0), (0.25, 4.0), (4.0, 0.25)])
def test_every_move_follows_an_edge(g12, pq):
    starts = np.arange(g12.n, dtype=np.uint32)
    r = O.walk(g12, starts, 30, *pq, seed=1)
    check_walks(g12, starts, r["out"], 30)
    assert r["transitions"] == int(np.sum(r["out"][:, 1:] != SENT))


def test_every_move_follows_an_edge_weighted(g11w):
    starts = np.arange(g11w.n, dtype=np.uint32)
    r = O.walk(g11w, starts, 25, 1.0, 0.5, seed=2)
    check_walks(g11w, starts, r["out"], 25)


def test_isolated_starts_give_sentinel_rows(g12):
    iso = np.nonzero(g12.degree() == 0)[0].astype(np.uint32)
    assert len(iso) > 0
    r = O.walk(g12, iso[:50], 10, 0.5, 2.0, seed=3)
    assert np.all(r["out"][:, 1:] == SENT)
    assert r["transitions"] == 0


def test_dead_end_in_directed_graph():
    # 0 -> 1 -> 2, nothing leaves 2: the walk stops there
    g = O.CSR(np.array([0, 1, 2, 2], dtype=np.uint64), np.array([1, 2], dtype=np.uint32))
    r = O.walk(g, np.array([0], dtype=np.uint32), 5, 1.0, 1.0, seed=1)
    assert r["out"].tolist() == [[0, 1, 2, SENT, SENT, SENT]]


def test_deterministic_and_thread_independent(g11w):
    starts = np.arange(g11w.n, dtype=np.uint32)
    a = O.walk(g11w, starts, 20, 0.25, 4.0, seed=9, nthreads=1)["out"]
    b = O.walk(g11w, starts, 20, 0.25, 4.0, seed=9, nthreads=8)["out"]
    c = O.walk(g11w, starts, 20, 0.25, 4.0, seed=10, nthreads=8)["out"]
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_walk_ids_select_the_random_stream(g12):
    # walk i with id walk_base + i equals the same walk run alone with that id
    starts = (np.arange(200, dtype=np.uint32) * 7) % g12.n
    full = O.walk(g12, starts, 15, 0.5, 2.0, seed=4, walk_base=1000)["out"]
    wids = np.arange(1000, 1200, dtype=np.uint64)
    pick = [3, 77, 150]
    part = O.walk(g12, starts[pick], 15, 0.5, 2.0, seed=4, wids=wids[pick])["out"]
    assert np.array_equal(full[pick], part)


def test_counts_and_checksum_definition(g12):
    starts = np.arange(0, g12.n, 5, dtype=np.uint32)
    seed, L, base = 11, 12, 500
    r = O.walk(g12, starts, L, 0.5, 2.0, seed=seed, walk_base=base, want_counts=True)
    out = r["out"]
    vals = out[out != SENT]
    assert np.array_equal(r["cnt"], np.bincount(vals, minlength=g12.n).astype(np.uint32))
    assert r["cnt"].sum() == len(starts) + r["transitions"]
    want = O.checksum_of(out, seed, np.arange(base, base + len(starts)))
    assert r["checksum"] == want


def test_checksum_is_chunking_invariant(g12):
    starts = np.tile(np.arange(g12.n, dtype=np.uint32), 2)
    full = O.walk(g12, starts, 20, 2.0, 0.5, seed=5, want_out=False, want_counts=True)
    cs, cnt = 0, np.zeros(g12.n, dtype=np.uint64)
    for lo in range(0, len(starts), 1500):
        hi = min(lo + 1500, len(starts))
        part = O.walk(g12, starts[lo:hi], 20, 2.0, 0.5, seed=5, walk_base=lo,
                      want_out=False, want_counts=True)
        cs = (cs + part["checksum"]) & 0xFFFFFFFFFFFFFFFF
        cnt += part["cnt"]
    assert cs == full["checksum"]
    assert np.array_equal(cnt, full["cnt"].astype(np.uint64))


def test_bad_arguments_rejected(g12):
    with pytest.raises(ValueError):
        O.walk(g12, np.array([0], dtype=np.uint32), 5, 0.3, 2.0, seed=1)
    with pytest.raises(ValueError):
        O.walk(g12, np.array([g12.n], dtype=np.uint32), 5, 0.5, 2.0, seed=1)


def test_cost_model_counts_moves(g12):
    starts = np.arange(0, g12.n, 3, dtype=np.uint32)
    wids = np.arange(len(starts), dtype=np.uint64)
    b, s, h = O.walk_cost(g12, starts, wids, 10, 0.5, 2.0, seed=1)
    r = O.walk(g12, starts, 10, 0.5, 2.0, seed=1, wids=wids)
    assert s == r["transitions"]
    # at least one 64-byte segment and the 4-byte output per move
    assert b >= s * (64 + 4)
    assert 0 <= h <= s


def test_visit_profile_buckets_by_hand():
    # star with centre 0 of degree 7 and a separate edge 8-9; vertex 10 isolated
    edges = [(0, i) for i in range(1, 8)] + [(8, 9)]
    g = O.CSR.from_edges(11, edges)
    cnt = np.array([10, 1, 1, 1, 1, 1, 1, 1, 4, 4, 3], dtype=np.uint32)
    verts, visits = O.visit_profile(g, cnt, 3, 4)
    # degree 0 -> bucket 0, degree 1 -> bucket 1 ((0, 3]), degree 7 -> bucket 3 (last: (6, 9] and above)
    assert verts.tolist() == [1, 9, 0, 1]
    assert visits.tolist() == [3, 15, 0, 10]
    verts, visits = O.visit_profile(g, cnt, 1, 8)
    assert verts.tolist() == [1, 9, 0, 0, 0, 0, 0, 1] and visits.tolist() == [3, 15, 0, 0, 0, 0, 0, 10]
