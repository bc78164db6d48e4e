"""Continuous-batching server: every result equals the oracle's walk of the
same request (walk ids 0.., the request's own seed), alone or in any mix."""
import time

import numpy as np
import pytest

import oracle as O
import paper_1805_00280_amd as P
from gpuhelp import gpu_graph_from_oracle, gpu_walk, oracle_rmat, say, torch_cuda

pytestmark = pytest.mark.gpu

PQ = [0.25, 0.5, 1.0, 2.0, 4.0]


@pytest.fixture(scope="module")
def graph():
    torch_cuda()
    og = oracle_rmat(13, 16, 0.57, 0.19, 0.19, 13, False)
    return og, gpu_graph_from_oracle(og, d_rule=64)


def requests(n_nodes, count, seed, max_size=5000):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        size = int(rng.integers(1, max_size))
        out.append(dict(starts=rng.integers(0, n_nodes, size=size).astype(np.uint32),
                        L=int(rng.choice([5, 20, 40])), p=float(rng.choice(PQ)), q=float(rng.choice(PQ)),
                        seed=int(rng.integers(0, 2**62))))
    return out


def wait_all(srv, tickets, timeout=60):
    t0 = time.time()
    done = {}
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.001)
    return done


def test_mix_equals_oracle_and_alone(graph):
    og, g = graph
    reqs = requests(og.n, 40, 1)
    srv = P.Server(g, pool_bytes=64 << 20, chunk_walks=700, max_inflight=16)
    tickets = [srv.submit(r["starts"], r["L"], r["p"], r["q"], r["seed"]) for r in reqs]
    done = wait_all(srv, tickets)
    for r, t in zip(reqs, tickets):
        got = srv.result_tensor(done[t])
        want = O.walk(og, r["starts"], r["L"], r["p"], r["q"], r["seed"], d_rule=64, nthreads=16)["out"]
        assert np.array_equal(got, want)
        alone = gpu_walk(g, r["starts"], r["L"], r["p"], r["q"], r["seed"])
        assert np.array_equal(got, alone)
        res = done[t]
        assert res.submit_ns <= res.start_ns <= res.done_ns
        srv.release(t)
    assert srv.stats() == (0, 0, 0)
    srv.close()


def test_mix_with_fn_approx_requests(graph):
    # exact and FN-Approx requests in one mix: each equals the oracle's rule for it
    og, g = graph
    reqs = requests(og.n, 24, 3)
    for i, r in enumerate(reqs):
        r["approx_t"] = (0, 30, 1000)[i % 3]
    srv = P.Server(g, pool_bytes=64 << 20, chunk_walks=700, max_inflight=16)
    tickets = [srv.submit(r["starts"], r["L"], r["p"], r["q"], r["seed"], approx_t=r["approx_t"]) for r in reqs]
    done = wait_all(srv, tickets)
    changed = 0
    for r, t in zip(reqs, tickets):
        got = srv.result_tensor(done[t])
        want = O.walk(og, r["starts"], r["L"], r["p"], r["q"], r["seed"], d_rule=64, nthreads=16,
                      approx_t=r["approx_t"])["out"]
        assert np.array_equal(got, want), r["approx_t"]
        if r["approx_t"]:
            exact = O.walk(og, r["starts"], r["L"], r["p"], r["q"], r["seed"], d_rule=64, nthreads=16)["out"]
            changed += int((exact != want).any(axis=1).sum())
        srv.release(t)
    assert changed > 0
    srv.close()


def test_tiny_pool_queues_and_admits_as_memory_frees(graph):
    og, g = graph
    # room for about two requests at a time: the rest wait for releases
    reqs = [dict(starts=np.arange(i * 100, i * 100 + 3000, dtype=np.uint32) % og.n, L=40, p=0.5, q=2.0, seed=i)
            for i in range(8)]
    per = 3000 * 4 + 3000 * 41 * 4
    srv = P.Server(g, pool_bytes=2 * (per + 4096) + 2 * 2**20, chunk_walks=512)
    tickets = [srv.submit(r["starts"], r["L"], r["p"], r["q"], r["seed"]) for r in reqs]
    say(f"[server] stats after submit {srv.stats()}")
    finished = 0
    t0 = time.time()
    while finished < len(tickets):
        for i, t in enumerate(tickets):
            if t is None:
                continue
            r = srv.poll(t)
            if r is not None:
                got = srv.result_tensor(r)
                want = O.walk(og, reqs[i]["starts"], 40, 0.5, 2.0, reqs[i]["seed"], d_rule=64)["out"]
                assert np.array_equal(got, want)
                srv.release(t)
                tickets[i] = None
                finished += 1
        assert time.time() - t0 < 60
        time.sleep(0.001)
    srv.close()


def test_errors(graph):
    og, g = graph
    srv = P.Server(g, pool_bytes=8 << 20)
    with pytest.raises(P.N2VError) as e:
        srv.submit(np.zeros(200000, dtype=np.uint32), 80, 1.0, 1.0, 1)
    assert e.value.code == -6  # ETOOBIG
    with pytest.raises(P.N2VError) as e:
        srv.submit(np.array([og.n], dtype=np.uint32), 5, 1.0, 1.0, 1)
    assert e.value.code == -1
    with pytest.raises(P.N2VError) as e:
        srv.submit(np.array([0], dtype=np.uint32), 5, 0.3, 1.0, 1)
    assert e.value.code == -1
    with pytest.raises(P.N2VError) as e:
        srv.poll(12345)
    assert e.value.code == -7
    t = srv.submit(np.array([1, 2, 3], dtype=np.uint32), 5, 1.0, 1.0, 1)
    wait_all(srv, [t])
    srv.release(t)
    with pytest.raises(P.N2VError):
        srv.release(t)
    srv.close()


def test_server_with_pair_sketches_from_garbage_memory():
    # sketch memory attached with arbitrary contents starts cleared, and the server (which keeps
    # sketches across ticks) returns the oracle's walks; the graph has many hubs (d_rule 40)
    import ctypes as C
    import torch
    torch_cuda()
    og = oracle_rmat(13, 16, 0.65, 0.15, 0.15, 5, False)
    g = gpu_graph_from_oracle(og, d_rule=40)
    b = C.c_size_t()
    assert P.lib().n2v_graph_memo_bytes(g._h, C.byref(b)) == 0 and b.value > 0
    buf = torch.full((b.value,), 0x37, dtype=torch.uint8, device="cuda")
    assert P.lib().n2v_graph_set_memo(g._h, C.c_void_p(buf.data_ptr()), b.value) == 0
    deg = og.degree()
    hubs = np.argsort(deg)[-64:].astype(np.uint32)
    reqs = [dict(starts=np.concatenate([np.repeat(hubs, 8), np.arange(i * 300, (i + 1) * 300, dtype=np.uint32)]),
                 L=20, p=float(PQ[i % 5]), q=float(PQ[(i * 2) % 5]), seed=1000 + i) for i in range(6)]
    srv = P.Server(g, pool_bytes=64 << 20, chunk_walks=700, max_inflight=8)
    tickets = [srv.submit(r["starts"], r["L"], r["p"], r["q"], r["seed"]) for r in reqs]
    done = wait_all(srv, tickets)
    for r, t in zip(reqs, tickets):
        got = srv.result_tensor(done[t])
        want = O.walk(og, r["starts"], r["L"], r["p"], r["q"], r["seed"], d_rule=40, nthreads=16)["out"]
        assert np.array_equal(got, want)
        srv.release(t)
    srv.close()
    assert P.lib().n2v_graph_set_memo(g._h, None, 0) == 0
    del buf


def test_live_server_blocks_memo_changes_and_destroy():
    # while a server holds the graph, attaching or detaching sketch memory and destroying the
    # graph return N2V_EINVAL and change nothing; after the server is gone all three work
    import ctypes as C
    import torch
    torch_cuda()
    og = oracle_rmat(12, 16, 0.65, 0.15, 0.15, 3, False)
    g = gpu_graph_from_oracle(og, d_rule=40)
    g.attach_memo()
    memo_before = g.memo
    srv = P.Server(g, pool_bytes=32 << 20, chunk_walks=512, max_inflight=4)
    b = C.c_size_t()
    assert P.lib().n2v_graph_memo_bytes(g._h, C.byref(b)) == 0
    other = torch.zeros(b.value, dtype=torch.uint8, device="cuda")
    assert P.lib().n2v_graph_set_memo(g._h, C.c_void_p(other.data_ptr()), b.value) == -1
    assert b"server" in P.lib().n2v_last_error()
    assert P.lib().n2v_graph_set_memo(g._h, None, 0) == -1
    assert P.lib().n2v_graph_set_memo_min(g._h, C.c_void_p(other.data_ptr()), b.value, 100) == -1
    assert P.lib().n2v_graph_destroy(g._h) == -1
    with pytest.raises(P.N2VError) as e:
        g.attach_memo()
    assert e.value.code == -1 and g.memo is memo_before
    starts = np.arange(0, og.n, 3, dtype=np.uint32)
    t = srv.submit(starts, 15, 0.5, 2.0, 21)
    done = wait_all(srv, [t])
    want = O.walk(og, starts, 15, 0.5, 2.0, 21, d_rule=40, nthreads=16)["out"]
    assert np.array_equal(srv.result_tensor(done[t]), want)
    srv.release(t)
    srv.close()
    assert P.lib().n2v_graph_set_memo(g._h, C.c_void_p(other.data_ptr()), b.value) == 0
    assert P.lib().n2v_graph_set_memo(g._h, None, 0) == 0
    g.close()
    del other


@pytest.mark.timeout(900)
def test_serving_workload_at_size():
    # the serving workload as the bench runs it: the R-MAT scale-22 graph resident with pair
    # sketches, a 24 GiB pool, 65536-walk chunks, 64 chunks and 2^19 walks per tick, and a
    # Philox-drawn request set that includes two 2^20-walk requests, all submitted together.
    # Every result equals the same request walked alone, and the oracle on sampled rows (all
    # rows of requests up to 2048 walks)
    import torch
    from paper_1805_00280_amd import workloads as WL
    from gpuhelp import u32
    torch_cuda()
    w = WL.C4
    g = P.Graph.from_rmat(*w.rmat_args(), weighted=False, device="cuda")
    g.attach_memo()
    og = oracle_rmat(*w.rmat_args(), False)
    assert np.array_equal(u32(g.adj), og.adj)
    reqs = [WL.serving_request(j, w.n) for j in range(14)]
    reqs += [WL.serving_request(100, w.n, size=1 << 20), WL.serving_request(101, w.n, size=1 << 20)]
    say(f"[c4] sizes {[len(r['starts']) for r in reqs]}")
    srv = P.Server(g, pool_bytes=24 << 30, chunk_walks=65536, max_inflight=64, tick_walks=1 << 19)
    tickets = [srv.submit(r["starts"], r["L"], r["p"], r["q"], r["seed"]) for r in reqs]
    done = wait_all(srv, tickets, timeout=300)
    rng = np.random.default_rng(9)
    for r, t in zip(reqs, tickets):
        got = srv.result_tensor(done[t])
        srv.release(t)
        n = len(r["starts"])
        alone = gpu_walk(g, r["starts"], r["L"], r["p"], r["q"], r["seed"])
        assert np.array_equal(got, alone), f"request of {n} walks differs from the same request alone"
        idx = np.arange(n) if n <= 2048 else np.sort(rng.choice(n, size=1024, replace=False))
        want = O.walk(og, r["starts"][idx], r["L"], r["p"], r["q"], r["seed"], wids=idx.astype(np.uint64),
                      nthreads=16)["out"]
        assert np.array_equal(got[idx], want), f"request of {n} walks differs from the oracle"
    say(f"[c4] {len(reqs)} requests equal alone and in the mix, and the oracle on sampled rows")
    srv.close()
    g.detach_memo()
