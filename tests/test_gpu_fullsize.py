"""Full-size workloads in the launch configuration bench.py times: every walk
of the workload on the device, seeded samples of rows checked against the
oracle walking its own copy of the graph, and the persistent form checked
against the plain form on every row."""
import numpy as np
import pytest

import oracle as O
import paper_1805_00280_amd as P
from paper_1805_00280_amd import workloads as WL
from gpuhelp import first_mismatch, oracle_rmat, say, torch_cuda, u32

pytestmark = pytest.mark.gpu


def _run(w, sample, attach_memo, approx_t=0):
    torch = torch_cuda()
    say(f"[full] {w.name}: device graph")
    g = P.Graph.from_rmat(*w.rmat_args(), weighted=w.weighted, device="cuda")
    if attach_memo:
        g.attach_memo()
    say(f"[full] {w.name}: oracle graph")
    og = oracle_rmat(*w.rmat_args(), w.weighted)
    assert np.array_equal(g.off.cpu().numpy().view(np.uint64), og.off)
    assert np.array_equal(u32(g.adj), og.adj)
    starts = torch.arange(w.walks, dtype=torch.int64, device="cuda").remainder_(w.n).to(torch.int32)
    out = torch.empty((w.walks, w.L + 1), dtype=torch.int32, device="cuda")
    say(f"[full] {w.name}: persistent pass over {w.walks} walks")
    g.walk(starts, w.L, w.p, w.q, w.seed, out=out, approx_t=approx_t)
    torch.cuda.synchronize()
    g.check_starts()
    ids = w.sample_walk_ids(sample, seed=99)
    got = u32(out[torch.from_numpy(ids.astype(np.int64)).cuda()])
    say(f"[full] {w.name}: oracle on {len(ids)} sampled walks")
    want = O.walk(og, (ids % w.n).astype(np.uint32), w.L, w.p, w.q, w.seed, wids=ids, nthreads=16,
                  approx_t=approx_t)["out"]
    assert first_mismatch(got, want) is None, first_mismatch(got, want)
    say(f"[full] {w.name}: plain pass")
    out2 = torch.empty_like(out)
    g.walk(starts, w.L, w.p, w.q, w.seed, out=out2, mode=P.MODE_PLAIN, approx_t=approx_t)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    moves = int((out[:, 1:] != -1).sum().item())
    say(f"[full] {w.name}: {moves} moves, persistent == plain on every row")
    return moves


@pytest.mark.timeout(600)
def test_scale20_weighted_workload():
    # 2^16 seeded-random walks of the 10.5M against the oracle, every row plain == persistent
    assert _run(WL.C2, 1 << 16, False) > 0


@pytest.mark.timeout(900)
def test_scale24_skewed_workload():
    # 2^16 seeded-random walks of the 67.1M against the oracle, every row plain == persistent
    assert _run(WL.C3, 1 << 16, True) > 0


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,pq", [("skew5", (0.5, 2.0)), ("skew1.78", (2.0, 0.5))])
def test_paper_skew_workloads(name, pq):
    # the paper's most skewed family member and WeC-22's twin, at full size
    assert _run(WL.paper_family(name, *pq), 512, True) > 0


@pytest.mark.timeout(900)
def test_paper_skew5_fn_approx():
    # FN-Approx at the paper's threshold on its most skewed graph, full size
    assert _run(WL.skew(5.0, 2.0, 0.5), 512, True, approx_t=1000) > 0


def test_paper_families_against_table1():
    # order-of-magnitude targets: the paper's graphs came from another generator
    torch = torch_cuda()
    for name in ("skew1", "skew2", "skew3", "skew4", "skew5", "wec22", "er22", "er24"):
        w = WL.paper_family(name)
        g = P.Graph.from_rmat(*w.rmat_args(), weighted=False, device="cuda")
        dmax = int((g.off[1:] - g.off[:-1]).max().item())
        m_paper, d_paper = WL.PAPER_TABLE1[name]
        say(f"[table1] {name}: m={g.m} ({m_paper:.4g}), max degree {dmax} ({d_paper})")
        assert abs(g.m - m_paper) / m_paper < 0.01
        assert d_paper / 2 <= dmax <= 2 * d_paper
        del g
        torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", [P.MODE_PERSISTENT, P.MODE_PLAIN])
def test_counts_workload_shape(mode):
    # the scale-27 counts workload's parameters (p=2, q=1/2, r=1, L=80, chunks
    # through walk_base) on a scale-16 graph, against the oracle's counts and checksum
    torch = torch_cuda()
    w = WL.C5
    scale = 16
    og = oracle_rmat(scale, 16, w.a, w.b, w.c, scale, False)
    g = P.Graph.from_rmat(scale, 16, w.a, w.b, w.c, scale, device="cuda")
    n = 1 << scale
    ref = O.walk(og, np.arange(n, dtype=np.uint32), w.L, w.p, w.q, w.seed, want_out=False, want_counts=True,
                 nthreads=16)
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    chunk = 10000
    for lo in range(0, n, chunk):
        hi = min(lo + chunk, n)
        st = torch.arange(lo, hi, dtype=torch.int32, device="cuda")
        g.walk_counts(st, w.L, w.p, w.q, w.seed, cnt, cs, walk_base=lo, mode=mode)
    torch.cuda.synchronize()
    assert np.array_equal(u32(cnt), ref["cnt"])
    assert int(cs.cpu().numpy().view(np.uint64)[0]) == ref["checksum"]


@pytest.mark.timeout(1200)
def test_scale27_counts_workload():
    # the counts workload at its own size: 4.2G directed entries (u64 offsets, rows past entry
    # 2^31), device CSR byte-equal to the oracle's; then the top 2^16 walk ids of the 2^27
    # (walk_base 2^27 - 2^16, counter words at the top of the 32-bit range) against the oracle:
    # visit counts, checksum and rows, with pair sketches on the highest-degree rows
    torch = torch_cuda()
    w = WL.C5
    say(f"[c5] {w.name}: device graph")
    g = P.Graph.from_rmat(*w.rmat_args(), weighted=False, device="cuda")
    # 2^32 directed keys generated, 4.22G entries after de-duplication: offsets past 2^31
    assert (1 << 31) < g.m < (1 << 32)
    memo = g.attach_memo(budget=24 << 30)
    say(f"[c5] m={g.m}, sketches {memo / 2**30:.1f} GiB for rows of degree >= {g.memo_min_degree}")
    say(f"[c5] oracle graph")
    og = O.rmat_csr(*w.rmat_args(), weighted=False, nthreads=16)
    assert og.m == g.m
    assert np.array_equal(g.off.cpu().numpy().view(np.uint64), og.off)
    step = 1 << 28
    for lo in range(0, og.m, step):
        hi = min(lo + step, og.m)
        assert np.array_equal(u32(g.adj[lo:hi]), og.adj[lo:hi]), (lo, hi)
    say(f"[c5] CSR byte-equal")
    k = 1 << 16
    base = w.walks - k
    st = torch.arange(base, w.walks, dtype=torch.int64, device="cuda").remainder_(w.n).to(torch.int32)
    cnt = torch.zeros(w.n, dtype=torch.int32, device="cuda")
    cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.empty((k, w.L + 1), dtype=torch.int32, device="cuda")
    say(f"[c5] walks [{base}, {w.walks}) on the device")
    g.walk_counts(st, w.L, w.p, w.q, w.seed, cnt, cs, walk_base=base, out=out)
    torch.cuda.synchronize()
    g.check_starts()
    say(f"[c5] oracle on the same walks")
    ref = O.walk(og, (np.arange(base, w.walks, dtype=np.uint64) % w.n).astype(np.uint32), w.L, w.p, w.q, w.seed,
                 walk_base=base, want_counts=True, nthreads=16)
    got = u32(out)
    assert first_mismatch(got, ref["out"]) is None, first_mismatch(got, ref["out"])
    assert np.array_equal(u32(cnt), ref["cnt"])
    assert int(cs.cpu().numpy().view(np.uint64)[0]) == ref["checksum"]
    say(f"[c5] {ref['transitions']} moves: rows, counts and checksum equal the oracle's")
    # a mid-range chunk reaches more of the graph (its starts have edges more often)
    base2, k2 = (1 << 26) + 12345, 4096
    st2 = torch.arange(base2, base2 + k2, dtype=torch.int32, device="cuda")
    out2 = g.walk(st2, w.L, w.p, w.q, w.seed, walk_base=base2)
    torch.cuda.synchronize()
    ref2 = O.walk(og, np.arange(base2, base2 + k2, dtype=np.uint32), w.L, w.p, w.q, w.seed, walk_base=base2,
                  nthreads=16)
    assert first_mismatch(u32(out2), ref2["out"]) is None, first_mismatch(u32(out2), ref2["out"])
    say(f"[c5] mid-range chunk: {ref2['transitions']} moves equal the oracle's")
