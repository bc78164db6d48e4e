"""GPU walks against the oracle: bit-exact on the same seeds."""
import itertools

import numpy as np
import pytest

import oracle as O
import paper_1805_00280_amd as P
from paper_1805_00280_amd import workloads as WL
from gpuhelp import (first_mismatch, gpu_graph_from_oracle, gpu_walk, oracle_rmat, oracle_walk, say,
                     starts_tensor, torch_cuda, u32)

pytestmark = pytest.mark.gpu

SKEW = (0.65, 0.15, 0.15)
DEF = (0.57, 0.19, 0.19)


@pytest.fixture(scope="module")
def c1():
    torch_cuda()
    w = WL.C1
    og = oracle_rmat(*w.rmat_args(), w.weighted)
    return w, og, gpu_graph_from_oracle(og)


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN])
def test_scale12_workload_full_parity(c1, mode):
    w, og, g = c1
    say(f"[walk] {w.name} mode={mode} walks={w.walks}")
    starts = w.starts()
    want = oracle_walk(og, starts, w.L, w.p, w.q, w.seed)
    got = gpu_walk(g, starts, w.L, w.p, w.q, w.seed, mode=mode)
    assert first_mismatch(got, want) is None, first_mismatch(got, want)


@pytest.mark.parametrize("opts", [
    dict(t_wave=0), dict(t_wave=16), dict(t_wave=1024), dict(sparse_ratio=1), dict(sparse_ratio=100000),
    dict(t_sparse=0), dict(waves_per_cu=4), dict(t_wave=0, sparse_ratio=1, waves_per_cu=1),
    dict(mode=P.MODE_PLAIN, t_wg=0), dict(mode=P.MODE_PLAIN, t_wg=0, sparse_ratio=100000),
    dict(mode=P.MODE_PLAIN, t_wg=1 << 31),
    dict(search_ratio=0), dict(search_ratio=0xFFFFFFFF), dict(search_ratio=0, sparse_ratio=100000),
    dict(mode=P.MODE_PLAIN, search_ratio=0, sparse_ratio=100000),
])
def test_execution_options_do_not_change_results(opts):
    torch_cuda()
    og = oracle_rmat(11, 16, *SKEW, 111, False)
    g = gpu_graph_from_oracle(og, d_rule=48)
    starts = np.tile(np.arange(og.n, dtype=np.uint32), 2)
    say(f"[walk] exec opts {opts}")
    want = oracle_walk(og, starts, 40, 0.25, 4.0, 77, d_rule=48)
    got = gpu_walk(g, starts, 40, 0.25, 4.0, 77, **opts)
    assert first_mismatch(got, want) is None, first_mismatch(got, want)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("d_rule,a_cap", [(0, 1024), (16, 1024), (0xFFFFFFFF, 1024), (1024, 1), (64, 2),
                                          (0xFFFFFFFF, 1)])
def test_rule_parameters(weighted, d_rule, a_cap):
    torch_cuda()
    og = oracle_rmat(10, 16, *SKEW, 10, weighted)
    g = gpu_graph_from_oracle(og, d_rule=d_rule, a_cap=a_cap)
    starts = np.arange(og.n, dtype=np.uint32)
    p, q = (1.0, 0.5) if weighted else (0.5, 2.0)
    say(f"[walk] rule d_rule={d_rule} a_cap={a_cap} weighted={weighted}")
    for mode in (P.MODE_PERSISTENT, P.MODE_PLAIN):
        want = oracle_walk(og, starts, 30, p, q, 5, d_rule=d_rule, a_cap=a_cap)
        got = gpu_walk(g, starts, 30, p, q, 5, mode=mode)
        assert first_mismatch(got, want) is None, (mode, first_mismatch(got, want))


@pytest.mark.parametrize("p,q", list(itertools.product([0.25, 0.5, 1.0, 2.0, 4.0], repeat=2)))
def test_all_p_q(p, q):
    # the plain form of a small superstep hands a lane's rejection chain to its
    # wavefront after 16 attempts: low acceptance (large 1/p against 1/q) makes
    # such chains common
    torch_cuda()
    og = oracle_rmat(10, 16, *SKEW, 3, False)
    g = gpu_graph_from_oracle(og, d_rule=32)
    starts = np.tile(np.arange(og.n, dtype=np.uint32), 4)
    want = oracle_walk(og, starts, 20, p, q, 9, d_rule=32)
    for mode in (P.MODE_PERSISTENT, P.MODE_PLAIN):
        got = gpu_walk(g, starts, 20, p, q, 9, mode=mode)
        assert first_mismatch(got, want) is None, (mode, first_mismatch(got, want))


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN])
@pytest.mark.parametrize("pq", [(1.0, 0.5), (0.25, 4.0), (4.0, 0.25)])
def test_weighted_with_hubs(mode, pq):
    torch_cuda()
    og = oracle_rmat(13, 16, *SKEW, 13, True)
    g = gpu_graph_from_oracle(og, d_rule=100)
    starts = np.arange(og.n, dtype=np.uint32)
    say(f"[walk] weighted hubs mode={mode} pq={pq}")
    want = oracle_walk(og, starts, 25, *pq, 31, d_rule=100)
    got = gpu_walk(g, starts, 25, *pq, 31, mode=mode)
    assert first_mismatch(got, want) is None, first_mismatch(got, want)


def _two_hub_graph():
    # hub 0 adjacent to every other vertex (degree beyond the 128 x 512 entries
    # one wavefront keeps chunk sums for), hub 1 to every third vertex, and a
    # sparse random layer so that low-degree vertices have common neighbours
    n = 70_000
    rng = np.random.default_rng(7)
    edges = [(0, v) for v in range(1, n)] + [(1, v) for v in range(3, n, 3)]
    a = rng.integers(2, n, size=60_000)
    b = rng.integers(2, n, size=60_000)
    edges += list(zip(a.tolist(), b.tolist()))
    return O.CSR.from_edges(n, edges)


def test_big_hubs_dense_and_sparse_paths():
    torch_cuda()
    og = _two_hub_graph()
    assert og.degree().max() > 512 * 128
    g = gpu_graph_from_oracle(og, d_rule=64)
    starts = np.concatenate([np.repeat(np.arange(6, dtype=np.uint32), 40),
                             np.arange(2, 2000, dtype=np.uint32)])
    want = oracle_walk(og, starts, 12, 0.5, 2.0, 3, d_rule=64)
    for ratio in (1, 100000):
        say(f"[walk] big hubs ratio={ratio}")
        got = gpu_walk(g, starts, 12, 0.5, 2.0, 3, sparse_ratio=ratio)
        assert first_mismatch(got, want) is None, first_mismatch(got, want)
        for search in (0, 0xFFFFFFFF):
            say(f"[walk] big hubs ratio={ratio} search_ratio={search}")
            got = gpu_walk(g, starts, 12, 0.5, 2.0, 3, sparse_ratio=ratio, search_ratio=search)
            assert first_mismatch(got, want) is None, first_mismatch(got, want)
        # plain form, every dense hub move evaluated by a whole workgroup
        say(f"[walk] big hubs ratio={ratio} workgroup class")
        got = gpu_walk(g, starts, 12, 0.5, 2.0, 3, sparse_ratio=ratio, mode=P.MODE_PLAIN, t_wg=0)
        assert first_mismatch(got, want) is None, first_mismatch(got, want)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("memo", [0, 1])
def test_workgroup_hub_class(weighted, memo):
    # the plain form hands dense hub moves above t_wg to whole workgroups: the segments of N(v)
    # are split among its wavefronts, and the located segment's tiles are taken four at a time
    torch = torch_cuda()
    og = oracle_rmat(13, 16, *SKEW, 13, weighted)
    g = gpu_graph_from_oracle(og, d_rule=100)
    if memo:
        g.attach_memo()
    deg = og.degree()
    hubs = np.argsort(deg)[-128:].astype(np.uint32)
    starts = np.concatenate([np.repeat(hubs, 16), np.arange(og.n, dtype=np.uint32)])
    pq = (1.0, 0.5) if weighted else (0.25, 4.0)
    want = oracle_walk(og, starts, 25, *pq, 31, d_rule=100)
    for t_wg, search in ((0, 2), (400, 2), (1 << 31, 2), (0, 0), (0, 0xFFFFFFFF)):
        say(f"[walk] workgroup class weighted={weighted} memo={memo} t_wg={t_wg} search={search}")
        got = gpu_walk(g, starts, 25, *pq, 31, mode=P.MODE_PLAIN, t_wg=t_wg, sparse_ratio=100000, memo=memo,
                       search_ratio=search)
        assert first_mismatch(got, want) is None, (t_wg, search, first_mismatch(got, want))
    if memo:
        torch.cuda.synchronize()
        n = check_sketch_rows(og, g.memo.cpu().numpy().view(np.uint16), 101)
        assert n > 100
        g.detach_memo()


def test_walk_base_selects_stream(c1):
    w, og, g = c1
    starts = w.starts(0, 3000)
    want = oracle_walk(og, starts, 15, w.p, w.q, w.seed, walk_base=123456)
    got = gpu_walk(g, starts, 15, w.p, w.q, w.seed, walk_base=123456)
    assert first_mismatch(got, want) is None


def test_edge_cases(c1):
    torch = torch_cuda()
    w, og, g = c1
    # no walks
    out = g.walk(starts_tensor(torch, np.zeros(0, np.uint32)), 5, 1.0, 1.0, 1)
    assert out.shape == (0, 6)
    # one move
    starts = w.starts(0, 500)
    assert first_mismatch(gpu_walk(g, starts, 1, w.p, w.q, 2), oracle_walk(og, starts, 1, w.p, w.q, 2)) is None
    # isolated starts
    iso = np.nonzero(og.degree() == 0)[0][:100].astype(np.uint32)
    got = gpu_walk(g, iso, 10, w.p, w.q, 2)
    assert np.all(got[:, 0] == iso) and np.all(got[:, 1:] == O.SENT)
    # start ids out of range: sentinel rows and a reported error
    bad = np.array([0, og.n + 5, 1], dtype=np.uint32)
    got = gpu_walk(g, bad, 4, w.p, w.q, 2)
    assert np.all(got[1, 1:] == O.SENT)
    assert first_mismatch(got[[0, 2]], oracle_walk(og, bad[[0, 2]], 4, w.p, w.q, 2, wids=[0, 2])) is None
    with pytest.raises(P.N2VError):
        g.check_starts()
    g.check_starts()  # the flag was cleared
    # bad p
    with pytest.raises(P.N2VError):
        g.walk(starts_tensor(torch, starts), 5, 0.3, 1.0, 1)


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN, "plain_wg"])
def test_directed_dead_end_and_tiny_graphs(mode):
    # dead ends reached by thread moves (d_rule 1024) and by hub moves (d_rule 0)
    kw = dict(mode=P.MODE_PLAIN, t_wg=0) if mode == "plain_wg" else dict(mode=mode)
    torch_cuda()
    g = O.CSR(np.array([0, 1, 2, 2], dtype=np.uint64), np.array([1, 2], dtype=np.uint32))
    for d_rule in (0, 1024):
        gg = gpu_graph_from_oracle(g, d_rule=d_rule)
        st3 = np.tile(np.array([0, 1, 2], dtype=np.uint32), 7)
        got = gpu_walk(gg, st3, 5, 1.0, 1.0, 1, **kw)
        assert first_mismatch(got, oracle_walk(g, st3, 5, 1.0, 1.0, 1, d_rule=d_rule)) is None, d_rule
    # a directed graph whose hubs lead into sinks: walks end at every superstep
    rng = np.random.default_rng(3)
    edges = sorted({(int(a), int(b)) for a, b in zip(rng.integers(0, 24, 1500), rng.integers(0, 40, 1500)) if a != b})
    off = np.zeros(41, dtype=np.uint64)
    for a, _ in edges:
        off[a + 1] += 1
    og = O.CSR(np.cumsum(off).astype(np.uint64), np.array([b for _, b in edges], dtype=np.uint32))
    for d_rule in (0, 32):
        gg = gpu_graph_from_oracle(og, d_rule=d_rule)
        starts = np.tile(np.arange(24, dtype=np.uint32), 40)
        want = oracle_walk(og, starts, 12, 0.5, 2.0, 9, d_rule=d_rule)
        assert (want == 0xFFFFFFFF).any()
        got = gpu_walk(gg, starts, 12, 0.5, 2.0, 9, **kw)
        assert first_mismatch(got, want) is None, (d_rule, first_mismatch(got, want))
    for edges, n in [([(0, 1)], 2), ([(0, i) for i in range(1, 40)], 40),
                     ([(a, b) for a in range(12) for b in range(a + 1, 12)], 12)]:
        og = O.CSR.from_edges(n, edges)
        for d_rule in (0, 1024):
            gg = gpu_graph_from_oracle(og, d_rule=d_rule)
            starts = np.tile(np.arange(n, dtype=np.uint32), 30)
            want = oracle_walk(og, starts, 15, 0.25, 4.0, 6, d_rule=d_rule)
            got = gpu_walk(gg, starts, 15, 0.25, 4.0, 6, **kw)
            assert first_mismatch(got, want) is None, (n, d_rule, first_mismatch(got, want))


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN, "plain_wg"])
def test_counts_and_checksum(mode):
    kw = dict(mode=P.MODE_PLAIN, t_wg=0) if mode == "plain_wg" else dict(mode=mode)
    torch = torch_cuda()
    og = oracle_rmat(12, 16, *DEF, 5, False)
    g = gpu_graph_from_oracle(og, d_rule=64)
    starts = np.tile(np.arange(og.n, dtype=np.uint32), 3)
    ref = O.walk(og, starts, 20, 2.0, 0.5, 5, d_rule=64, want_counts=True, nthreads=16)
    cnt = torch.zeros(og.n, dtype=torch.int32, device="cuda")
    cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    # three chunks with walk_base, counts accumulate
    for lo in range(0, len(starts), 5000):
        hi = min(lo + 5000, len(starts))
        g.walk_counts(starts_tensor(torch, starts[lo:hi]), 20, 2.0, 0.5, 5, cnt, cs, walk_base=lo, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(u32(cnt), ref["cnt"])
    assert int(cs.cpu().numpy().view(np.uint64)[0]) == ref["checksum"]
    # counts and walks together
    out = torch.empty((len(starts), 21), dtype=torch.int32, device="cuda")
    cnt.zero_()
    cs.zero_()
    g.walk_counts(starts_tensor(torch, starts), 20, 2.0, 0.5, 5, cnt, cs, out=out, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(u32(out), ref["out"])
    assert np.array_equal(u32(cnt), ref["cnt"])


def test_autotune_keeps_results(c1):
    w, og, g = c1
    best, ms = g.autotune(4096, 40, w.p, w.q)
    say(f"[tune] best={best.as_dict()} ms={ms:.3f}")
    assert ms > 0
    starts = w.starts(0, 8000)
    want = oracle_walk(og, starts, w.L, w.p, w.q, w.seed)
    got = gpu_walk(g, starts, w.L, w.p, w.q, w.seed)
    assert first_mismatch(got, want) is None


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN])
def test_pair_sketches_keep_results(mode):
    # many walks from the hubs traverse the same hub pairs again and again, so
    # most dense hub moves read a sketch written earlier in the same call
    torch_cuda()
    og = oracle_rmat(14, 16, *SKEW, 14, False)
    g = gpu_graph_from_oracle(og, d_rule=40)
    assert g.attach_memo() > 0
    deg = og.degree()
    hubs = np.argsort(deg)[-256:].astype(np.uint32)
    starts = np.concatenate([np.repeat(hubs, 64), np.arange(og.n, dtype=np.uint32)])
    want = oracle_walk(og, starts, 30, 0.25, 4.0, 8, d_rule=40)
    for rep in range(2):  # the second call starts from cleared sketches again
        say(f"[walk] sketches mode={mode} rep={rep}")
        got = gpu_walk(g, starts, 30, 0.25, 4.0, 8, mode=mode, sparse_ratio=100000)
        assert first_mismatch(got, want) is None, first_mismatch(got, want)
    got = gpu_walk(g, starts, 30, 0.25, 4.0, 8, mode=mode, memo=0)
    assert first_mismatch(got, want) is None
    g.detach_memo()


def sketch_segments(d, tile=512, segs=64):
    """Segment length and count of a hub row of degree d: tiles of 512 entries, grouped evenly into
    at most 64 segments."""
    nsub = -(-d // tile)
    G = -(-nsub // segs)
    return G * tile, -(-nsub // G)


def hint_shift(d):
    return max(0, int(d).bit_length() - 15)


def memo_segs(d):
    """Entries per array of a sketch row of a vertex of degree d: its segment count, rounded up to
    even (every row a whole number of 4-byte words)."""
    _, nsup = sketch_segments(int(d))
    return (nsup + 1) & ~1


def row_words(d, weighted):
    return (11 if weighted else 3) * memo_segs(d)


def sketch_bytes(deg, min_deg, weighted=False):
    """Sketch memory of the rows of degree >= min_deg: deg(v) rows of row_words(deg v) u16 each."""
    return sum(2 * int(d) * row_words(d, weighted) for d in deg[deg >= min_deg] if d > 0)


def check_sketch_rows(og, memo, min_deg, limit=6000, seed=1):
    """Every written pair-sketch row (v, index of t in N(v)) holds, per segment of N(v), one plus the
    number of its entries that are neighbours of t; start hints into N(t) at or below the lower
    bound of the segment's first entry and not below the end of the previous segment's matches; and
    one plus the number in the segment's first half (0 where unknown). Unwritten rows and entries
    are zero.  `memo` is the flat u16 sketch memory: the rows of each vertex of degree >= min_deg in
    vertex order, deg(v) rows of row_words(deg v) words each."""
    deg = og.degree()
    weighted = og.wt is not None
    hub = (deg >= min_deg) & (deg > 0)
    words = np.array([int(d) * row_words(d, weighted) if h else 0 for d, h in zip(deg, hub)], dtype=np.int64)
    hb = np.zeros(og.n + 1, dtype=np.int64)
    hb[1:] = np.cumsum(words)
    assert memo.shape[0] >= hb[-1]
    touched = []
    for v in np.nonzero(hub)[0]:
        block = memo[hb[v]:hb[v + 1]].reshape(int(deg[v]), row_words(deg[v], weighted))
        for pos in np.nonzero(block.any(axis=1))[0]:
            touched.append((int(v), int(pos)))
    rng = np.random.default_rng(seed)
    pick = touched if len(touched) <= limit else [touched[i] for i in rng.choice(len(touched), limit, replace=False)]
    hinted = halves = 0
    for v, pos in pick:
        nsp = memo_segs(deg[v])
        rw = row_words(deg[v], weighted)
        row = memo[hb[v] + pos * rw:hb[v] + (pos + 1) * rw]
        counts, hints, halfs = row[:nsp], row[nsp:2 * nsp], row[2 * nsp:3 * nsp]
        nv = og.row(v)
        t = int(nv[pos])
        nt = og.row(t)
        seglen, nsup = sketch_segments(int(deg[v]))
        com = np.isin(nv, nt, assume_unique=True)
        firsts = np.arange(0, len(nv), seglen)
        want = np.add.reduceat(com.astype(np.int64), firsts) + 1
        assert np.array_equal(counts[:nsup], want), (v, t, counts[:nsup], want)
        assert not counts[nsup:].any() and not hints[nsup:].any() and not halfs[nsup:].any()
        if weighted:
            # per segment: members' weight sum + 1, the same over the first half + 1, all
            # entries' weight sum, the same over the first half (0 where not written)
            sums = np.ascontiguousarray(row[3 * nsp:]).view(np.uint32).astype(np.int64)
            w = og.wt[int(og.off[v]):int(og.off[v + 1])].astype(np.int64)
            cw = np.add.reduceat(np.where(com, w, 0), firsts)
            wa = np.add.reduceat(w, firsts)
            cw1 = np.array([int(np.where(com, w, 0)[a:min(a + seglen // 2, len(nv))].sum()) for a in firsts])
            wa1 = np.array([int(w[a:min(a + seglen // 2, len(nv))].sum()) for a in firsts])
            for k, want_k in enumerate((cw + 1, cw1 + 1, wa, wa1)):
                part = sums[k * nsp:k * nsp + nsup]
                assert np.all((part == 0) | (part == want_k)), (v, t, k)
                assert not sums[k * nsp + nsup:(k + 1) * nsp].any()
            assert np.all(sums[0:nsup] == cw + 1) and np.all(sums[2 * nsp:2 * nsp + nsup] == wa)
        half = np.array([int(com[a:min(a + seglen // 2, len(nv))].sum()) for a in firsts]) + 1
        hv = halfs[:nsup].astype(np.int64)
        hknown = hv > 0
        halves += int(hknown.sum())
        assert np.array_equal(hv[hknown], half[hknown]), (v, t, hv, half)
        hs = hint_shift(len(nt))
        lb = np.searchsorted(nt, nv[firsts], side="left")
        ub_prev = np.concatenate([[0], np.searchsorted(nt, nv[firsts[1:] - 1], side="right")])
        h = hints[:nsup].astype(np.int64)
        known = h > 0
        hinted += int(known.sum())
        assert np.all((ub_prev >> hs)[known] <= h[known] - 1), (v, t)
        assert np.all(h[known] - 1 <= (lb >> hs)[known]), (v, t)
    assert hinted > 0 and halves > 0
    return len(touched)


@pytest.mark.parametrize("mode,t_wg,search", [(P.MODE_PERSISTENT, 65536, 2), (P.MODE_PLAIN, 65536, 2),
                                               (P.MODE_PLAIN, 0, 2), (P.MODE_PERSISTENT, 65536, 0),
                                               (P.MODE_PERSISTENT, 65536, 0xFFFFFFFF)])
def test_pair_sketch_contents(mode, t_wg, search):
    # the sketches written during a call (by forward merges and by the reverse pairs they also
    # count) hold exact per-segment common-neighbour counts
    import torch
    torch_cuda()
    og = oracle_rmat(14, 16, *SKEW, 14, False)
    g = gpu_graph_from_oracle(og, d_rule=40)
    g.attach_memo()
    deg = og.degree()
    hubs = np.argsort(deg)[-256:].astype(np.uint32)
    starts = np.concatenate([np.repeat(hubs, 16), np.arange(og.n, dtype=np.uint32)])
    got = gpu_walk(g, starts, 20, 0.25, 4.0, 8, mode=mode, sparse_ratio=100000, t_wg=t_wg, search_ratio=search)
    torch.cuda.synchronize()
    memo = g.memo.cpu().numpy().view(np.uint16)
    n = check_sketch_rows(og, memo, 41)
    say(f"[walk] sketches mode={mode}: {n} rows written")
    assert n > 1000
    want = oracle_walk(og, starts, 20, 0.25, 4.0, 8, d_rule=40)
    assert first_mismatch(got, want) is None
    g.detach_memo()


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN])
def test_pair_sketches_above_degree_threshold(mode):
    # with a memory budget below the full size, only rows of the highest-degree vertices keep
    # sketches; results are unchanged, and re-attaching the full size re-indexes the rows
    import torch
    torch_cuda()
    og = oracle_rmat(14, 16, *SKEW, 14, False)
    g = gpu_graph_from_oracle(og, d_rule=40)
    full = g.attach_memo()
    g.detach_memo()
    deg = og.degree()
    got_bytes = g.attach_memo(budget=full // 3)
    T = g.memo_min_degree
    assert full == sketch_bytes(deg, 41)
    assert 41 < T < 2 ** 20 and got_bytes == sketch_bytes(deg, T) <= full // 3
    # the threshold is the smallest that fits
    assert T - 1 <= 41 or sketch_bytes(deg, T - 1) > full // 3
    hubs = np.argsort(deg)[-256:].astype(np.uint32)
    starts = np.concatenate([np.repeat(hubs, 16), np.arange(og.n, dtype=np.uint32)])
    want = oracle_walk(og, starts, 20, 0.25, 4.0, 8, d_rule=40)
    say(f"[walk] sketches above degree {T} mode={mode}")
    got = gpu_walk(g, starts, 20, 0.25, 4.0, 8, mode=mode, sparse_ratio=4)
    assert first_mismatch(got, want) is None
    torch.cuda.synchronize()
    n = check_sketch_rows(og, g.memo.cpu().numpy().view(np.uint16), T)
    assert n > 100
    g.detach_memo()
    assert g.attach_memo() == full
    got = gpu_walk(g, starts, 20, 0.25, 4.0, 8, mode=mode, sparse_ratio=4)
    assert first_mismatch(got, want) is None
    torch.cuda.synchronize()
    assert check_sketch_rows(og, g.memo.cpu().numpy().view(np.uint16), 41) > 100
    g.detach_memo()
    assert g.attach_memo(budget=0) == 0


# ------------------------------------------------------------------ FN-Approx
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN, "plain_wg"])
def test_fn_approx_matches_oracle(weighted, mode):
    # moves at vertices above d_rule reached from vertices at or below it are
    # drawn from the static weights when the bound gap is below 1/T
    torch_cuda()
    og = oracle_rmat(13, 16, *SKEW, 13, False)
    if weighted:
        # weights in [1, 3], symmetric: a narrow range, so that the bounds meet
        src = np.repeat(np.arange(og.n, dtype=np.int64), og.degree().astype(np.int64))
        dst = og.adj.astype(np.int64)
        lo, hi = np.minimum(src, dst), np.maximum(src, dst)
        og = O.CSR(og.off, og.adj, (1 + (lo * 7 + hi * 13) % 3).astype(np.uint16))
    g = gpu_graph_from_oracle(og, d_rule=100)
    if not weighted:
        g.attach_memo()
    deg = og.degree()
    hubs = np.argsort(deg)[-64:].astype(np.uint32)
    starts = np.concatenate([np.repeat(hubs, 8), np.arange(og.n, dtype=np.uint32)])
    kw = dict(mode=P.MODE_PLAIN, t_wg=0) if mode == "plain_wg" else dict(mode=mode)
    cases = [((0.5, 2.0), 100), ((2.0, 0.5), 1000), ((0.25, 4.0), 30), ((4.0, 0.25), 300), ((1.0, 0.5), 1)]
    if weighted:
        cases = [((0.5, 2.0), 30), ((2.0, 0.5), 100), ((0.25, 1.0), 20)]
    for (p, q), T in cases:
        say(f"[approx] weighted={weighted} mode={mode} p={p} q={q} T={T}")
        want = oracle_walk(og, starts, 30, p, q, 17, d_rule=100, approx_t=T)
        exact = oracle_walk(og, starts, 30, p, q, 17, d_rule=100)
        assert (want != exact).any(axis=1).sum() > 100  # the rule is exercised
        got = gpu_walk(g, starts, 30, p, q, 17, approx_t=T, **kw)
        assert first_mismatch(got, want) is None, (p, q, T, first_mismatch(got, want))
    # threshold 0 is the exact rule
    got = gpu_walk(g, starts, 30, 0.5, 2.0, 17, approx_t=0, **kw)
    want = oracle_walk(og, starts, 30, 0.5, 2.0, 17, d_rule=100)
    assert first_mismatch(got, want) is None, first_mismatch(got, want)


def test_fn_approx_big_hubs_and_counts():
    torch = torch_cuda()
    og = _two_hub_graph()
    g = gpu_graph_from_oracle(og, d_rule=64)
    g.attach_memo()
    starts = np.concatenate([np.repeat(np.arange(6, dtype=np.uint32), 40), np.arange(2, 3000, dtype=np.uint32)])
    for T in (1000, 20000):
        want = oracle_walk(og, starts, 12, 0.5, 2.0, 3, d_rule=64, approx_t=T)
        for kw in (dict(), dict(sparse_ratio=100000, search_ratio=0), dict(mode=P.MODE_PLAIN, t_wg=0)):
            say(f"[approx] big hubs T={T} {kw}")
            got = gpu_walk(g, starts, 12, 0.5, 2.0, 3, approx_t=T, **kw)
            assert first_mismatch(got, want) is None, (T, kw, first_mismatch(got, want))
    ref = O.walk(og, starts, 12, 0.5, 2.0, 3, d_rule=64, approx_t=1000, want_out=False, want_counts=True,
                 nthreads=16)
    for mode in (P.MODE_PERSISTENT, P.MODE_PLAIN):
        cnt = torch.zeros(og.n, dtype=torch.int32, device="cuda")
        cs = torch.zeros(1, dtype=torch.int64, device="cuda")
        g.walk_counts(starts_tensor(torch, starts), 12, 0.5, 2.0, 3, cnt, cs, mode=mode, approx_t=1000)
        torch.cuda.synchronize()
        assert np.array_equal(u32(cnt), ref["cnt"])
        assert int(cs.cpu().numpy().view(np.uint64)[0]) == ref["checksum"]


def test_visit_profile_matches_oracle_and_degree_bias():
    # the paper's frequency-versus-degree study: mean visits per degree bucket
    torch = torch_cuda()
    og = oracle_rmat(14, 16, *DEF, 14, False)
    g = gpu_graph_from_oracle(og)
    starts = np.tile(np.arange(og.n, dtype=np.uint32), 4)
    cnt = torch.zeros(og.n, dtype=torch.int32, device="cuda")
    cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    g.walk_counts(starts_tensor(torch, starts), 80, 1.0, 1.0, 5, cnt, cs)
    for width, nb in ((50, 64), (1, 2048), (1000, 2)):
        verts, visits = g.visit_profile(cnt, width, nb)
        torch.cuda.synchronize()
        ov, oc = O.visit_profile(og, u32(cnt), width, nb)
        assert np.array_equal(verts.cpu().numpy(), ov) and np.array_equal(visits.cpu().numpy(), oc), width
    # first-order walks (p = q = 1) visit a vertex about in proportion to its degree
    ov, oc = O.visit_profile(og, u32(cnt), 20, 64)
    keep = ov[1:-1] >= 20
    mid = (np.arange(1, 63) * 20 - 10)[keep]
    mean = oc[1:-1][keep] / ov[1:-1][keep]
    assert np.corrcoef(mid, mean)[0, 1] > 0.95
    with pytest.raises(P.N2VError):
        g.visit_profile(cnt, 0, 8)
    with pytest.raises(P.N2VError):
        g.visit_profile(cnt, 10, 4096)


def test_uniform_weights_walk_like_unweighted():
    # all weights 7: the weighted kernels (weight scans, row totals) must draw
    # exactly what the unweighted ones draw, exact rule and FN-Approx
    torch_cuda()
    og = oracle_rmat(12, 16, *SKEW, 12, False)
    w7 = O.CSR(og.off, og.adj, np.full(og.m, 7, dtype=np.uint16))
    g0 = gpu_graph_from_oracle(og, d_rule=64)
    g7 = gpu_graph_from_oracle(w7, d_rule=64)
    starts = np.tile(np.arange(og.n, dtype=np.uint32), 2)
    for mode in (P.MODE_PERSISTENT, P.MODE_PLAIN):
        for T in (0, 50):
            say(f"[walk] uniform weights mode={mode} approx_t={T}")
            a = gpu_walk(g0, starts, 20, 0.5, 2.0, 9, approx_t=T, mode=mode)
            b = gpu_walk(g7, starts, 20, 0.5, 2.0, 9, approx_t=T, mode=mode)
            assert first_mismatch(b, a) is None, (mode, T, first_mismatch(b, a))
            want = oracle_walk(og, starts, 20, 0.5, 2.0, 9, d_rule=64, approx_t=T)
            assert first_mismatch(a, want) is None, (mode, T, first_mismatch(a, want))


def test_memo_min_refusal_leaves_the_graph_unchanged():
    # too few bytes for a lower threshold: N2V_ENOMEM, and the graph keeps its rows and
    # memory, so the next walks (which read sketches indexed by those rows) equal the oracle's
    import ctypes as C
    import torch
    torch_cuda()
    og = oracle_rmat(13, 16, *SKEW, 13, False)
    g = gpu_graph_from_oracle(og, d_rule=40)
    deg = og.degree()
    full = g.attach_memo()
    g.detach_memo()
    part = g.attach_memo(budget=full // 4)
    T = g.memo_min_degree
    assert part > 0 and T > 41
    # ask for every hub row (threshold 41) with only the partial size
    small = torch.zeros(part, dtype=torch.uint8, device="cuda")
    rc = P.lib().n2v_graph_set_memo_min(g._h, C.c_void_p(small.data_ptr()), part, 41)
    assert rc == -2, rc
    hubs = np.argsort(deg)[-128:].astype(np.uint32)
    starts = np.concatenate([np.repeat(hubs, 8), np.arange(og.n, dtype=np.uint32)])
    say(f"[walk] refused re-index (threshold {T} kept)")
    got = gpu_walk(g, starts, 20, 0.25, 4.0, 9)
    want = oracle_walk(og, starts, 20, 0.25, 4.0, 9, d_rule=40)
    assert first_mismatch(got, want) is None, first_mismatch(got, want)
    n = check_sketch_rows(og, g.memo.cpu().numpy().view(np.uint16), T)
    assert n > 50
    g.detach_memo()
    del small


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN])
def test_sketches_persist_across_calls_and_clear(mode):
    # sketches describe the graph only: a second call with other (p, q, seed) reuses what the
    # first filled and still equals the oracle; after n2v_graph_memo_clear every entry is unknown
    import torch
    torch_cuda()
    og = oracle_rmat(13, 16, *SKEW, 17, False)
    g = gpu_graph_from_oracle(og, d_rule=40)
    g.attach_memo()
    deg = og.degree()
    hubs = np.argsort(deg)[-128:].astype(np.uint32)
    starts = np.concatenate([np.repeat(hubs, 8), np.arange(og.n, dtype=np.uint32)])
    say(f"[walk] persisting sketches mode={mode}")
    for p, q, seed in [(0.25, 4.0, 1), (2.0, 0.5, 2), (1.0, 1.0, 3)]:
        got = gpu_walk(g, starts, 20, p, q, seed, mode=mode)
        want = oracle_walk(og, starts, 20, p, q, seed, d_rule=40)
        assert first_mismatch(got, want) is None, (p, q, first_mismatch(got, want))
    memo = g.memo.cpu().numpy().view(np.uint16)
    assert np.count_nonzero(memo) > 0
    assert check_sketch_rows(og, memo, 41) > 100
    g.memo_clear()
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(g.memo).item()) == 0
    got = gpu_walk(g, starts, 20, 0.5, 2.0, 4, mode=mode)
    assert first_mismatch(got, oracle_walk(og, starts, 20, 0.5, 2.0, 4, d_rule=40)) is None
    g.detach_memo()


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN])
def test_weighted_pair_sketches(mode):
    # weighted graphs keep sketches too (per-segment weight sums of the members of N(t) and of
    # all entries beside the counts): walks over several calls, which read the rows the earlier
    # ones wrote, equal the oracle's, and the rows hold exact sums
    import torch
    torch_cuda()
    og = oracle_rmat(13, 16, *SKEW, 23, True)
    g = gpu_graph_from_oracle(og, d_rule=40)
    assert g.attach_memo() > 0
    deg = og.degree()
    hubs = np.argsort(deg)[-128:].astype(np.uint32)
    starts = np.concatenate([np.repeat(hubs, 8), np.arange(og.n, dtype=np.uint32)])
    say(f"[walk] weighted sketches mode={mode}")
    for p, q, seed, opts in [(1.0, 0.5, 1, {}), (0.25, 4.0, 2, {"search_ratio": 0}), (2.0, 0.5, 3, {"sparse_ratio": 1})]:
        got = gpu_walk(g, starts, 20, p, q, seed, mode=mode, **opts)
        want = oracle_walk(og, starts, 20, p, q, seed, d_rule=40)
        assert first_mismatch(got, want) is None, (p, q, first_mismatch(got, want))
    torch.cuda.synchronize()
    n = check_sketch_rows(og, g.memo.cpu().numpy().view(np.uint16), 41)
    assert n > 100
    g.detach_memo()


@pytest.mark.parametrize("weighted", [False, True])
def test_plain_form_graph_replays(weighted):
    # a plain-form call whose arguments repeat is captured on its second
    # occurrence and replayed afterwards: every call, direct, capturing or
    # replayed, must match the oracle, also after the buffers' contents change,
    # on another stream, and after more distinct calls than the graph keeps
    torch = torch_cuda()
    og = oracle_rmat(12, 16, *SKEW, 21, weighted)
    g = gpu_graph_from_oracle(og, d_rule=64)
    g.attach_memo()
    pq = (1.0, 0.5) if weighted else (0.25, 4.0)
    L = 30
    opts = P.exec_opts(g, mode=P.MODE_PLAIN, t_wg=200)
    starts_a = np.tile(np.arange(og.n, dtype=np.uint32), 2)
    starts_b = np.random.default_rng(5).integers(0, og.n, len(starts_a)).astype(np.uint32)
    n = len(starts_a)
    st = starts_tensor(torch, starts_a)
    out = torch.empty((n, L + 1), dtype=torch.int32, device="cuda")
    ws = P._alloc(g.walk_workspace(n, L, opts), "cuda")
    side = torch.cuda.Stream()
    seeds = list(range(40, 50))  # more distinct calls than the graph keeps captured
    want = {(k, s): oracle_walk(og, src, L, *pq, s, d_rule=64)
            for k, src in (("a", starts_a), ("b", starts_b)) for s in seeds[:2]}
    plan = [("a", seeds[0])] * 3 + [("b", seeds[0])] * 2 + [("a", seeds[1])] * 2
    plan += [("a", s) for s in seeds for _ in range(2)] + [("b", seeds[1]), ("a", seeds[0])] * 2
    for k, (src, seed) in enumerate(plan):
        say(f"[walk] plain replay call {k}: starts {src} seed {seed} weighted={weighted}")
        stream = side if k % 3 == 2 else torch.cuda.current_stream()
        torch.cuda.synchronize()
        st.copy_(torch.from_numpy((starts_a if src == "a" else starts_b).view(np.int32)))
        out.fill_(-7)
        torch.cuda.synchronize()
        g.walk(st, L, *pq, seed, out=out, opts=opts, ws=ws, stream=stream)
        torch.cuda.synchronize()
        ref = want.get((src, seed))
        if ref is None:
            ref = want[(src, seed)] = oracle_walk(og, starts_a if src == "a" else starts_b, L, *pq, seed, d_rule=64)
        assert first_mismatch(u32(out), ref) is None, (k, src, seed, first_mismatch(u32(out), ref))
    # counts replayed the same way accumulate like direct calls
    cnt = torch.zeros(og.n, dtype=torch.int32, device="cuda")
    cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    st.copy_(torch.from_numpy(starts_a.view(np.int32)))
    for _ in range(3):
        g.walk_counts(st, L, *pq, seeds[0], cnt, cs, opts=opts, ws=ws)
    torch.cuda.synchronize()
    ref = O.walk(og, starts_a, L, *pq, seeds[0], d_rule=64, want_counts=True, nthreads=16)
    assert np.array_equal(u32(cnt), 3 * ref["cnt"].astype(np.uint32))
    assert int(cs.cpu().numpy().view(np.uint64)[0]) == (3 * ref["checksum"]) % (1 << 64)
