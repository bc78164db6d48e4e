"""The paper's synthetic graph families (Section 4.1) as generated here: names,
quadrant probabilities, and the edge-count reading checked against Table 1 on
the one family member small enough for the CPU oracle in a second."""
import numpy as np
import pytest

import oracle as O
from paper_1805_00280_amd import workloads as WL


def test_family_parameters():
    w = WL.paper_family("skew3")
    assert (w.scale, w.edge_factor, w.r, w.L, w.p, w.q) == (22, 50, 1, 80, 0.5, 2.0)
    d = 1.0 - w.a - w.b - w.c
    assert w.b == w.c == 0.25 and d == pytest.approx(3.0 * w.a)
    # WeC-22 is Skew-1.78 up to rounding of its quadrant probabilities
    s, c = WL.paper_family("skew1.78"), WL.paper_family("wec22")
    assert abs(s.a - c.a) < 1e-3 and (s.scale, s.edge_factor) == (c.scale, c.edge_factor)
    e = WL.paper_family("er26", 2.0, 0.5)
    assert (e.a, e.b, e.c, e.edge_factor, e.p, e.q) == (0.25, 0.25, 0.25, 5, 2.0, 0.5)
    assert e.name == "er26-p2-q0.5-r1-L80"
    for bad in ("skew", "er", "wec20.5", "c3", "skew-2"):
        with pytest.raises(ValueError):
            WL.paper_family(bad)


def test_er20_matches_table1():
    # Table 1: ER-20 has 10.5M edges and maximum degree 29; the symmetrized
    # reading (edge factor 5, both directions stored) reproduces both.
    w = WL.er(20)
    og = O.rmat_csr(*w.rmat_args(), weighted=False, nthreads=8)
    deg = np.diff(og.off.astype(np.int64))
    m_paper, dmax_paper = WL.PAPER_TABLE1["er20"]
    assert abs(og.m - m_paper) / m_paper < 0.01
    assert abs(int(deg.max()) - dmax_paper) <= 3
    assert abs(deg.mean() - 10.0) < 0.05


def test_wec20_matches_table1():
    # Table 1: WeC-20 has 104.8M edges and maximum degree 1053 (the paper's
    # generator is another one, so the degree is an order-of-magnitude target)
    w = WL.wec(20)
    og = O.rmat_csr(*w.rmat_args(), weighted=False, nthreads=8)
    deg = np.diff(og.off.astype(np.int64))
    m_paper, dmax_paper = WL.PAPER_TABLE1["wec20"]
    assert abs(og.m - m_paper) / m_paper < 0.005
    assert dmax_paper / 2 <= int(deg.max()) <= 2 * dmax_paper
    assert abs(deg.mean() - 100.0) < 0.1


def test_request_stream_philox_matches_the_reference_copy():
    # the input generator's vectorised Philox against the pure-Python copy
    from oracle.philox_ref import philox4x32
    rng = np.random.default_rng(2)
    c = rng.integers(0, 2**32, size=(4, 500), dtype=np.uint64)
    k0, k1 = 0x1234567, 0x89ABCDEF
    got = WL.philox_np(k0, k1, *c)
    for i in range(500):
        want = philox4x32((k0, k1), [int(x) for x in c[:, i]])
        assert [int(g[i]) for g in got] == want


def test_request_stream_shape():
    # sizes floor(2^(20U)) in [1, 2^20] (mean about (2^20 - 1) / (20 ln 2) = 75.6K), L in
    # {20, 40, 80}, p and q over five values, starts below n; the stream is reproducible
    n = 1 << 22
    reqs = [WL.serving_request(j, n) for j in range(200)]
    sizes = np.array([len(r["starts"]) for r in reqs])
    assert sizes.min() >= 1 and sizes.max() <= 1 << 20
    logs = np.log2(sizes + 1)
    assert 8.0 < logs.mean() < 12.0
    assert {r["L"] for r in reqs} == {20, 40, 80}
    assert {r["p"] for r in reqs} == {0.25, 0.5, 1.0, 2.0, 4.0} == {r["q"] for r in reqs}
    assert all(int(r["starts"].max()) < n for r in reqs)
    again = WL.serving_request(17, n)
    assert np.array_equal(again["starts"], reqs[17]["starts"]) and again["seed"] == reqs[17]["seed"]
    big = WL.serving_request(3, n, size=1 << 20)
    assert len(big["starts"]) == 1 << 20 and abs(big["starts"].mean() / n - 0.5) < 0.01
    t = WL.arrival_times(reqs, rate=100.0)
    assert np.all(np.diff(t) > 0) and 1.2 < t[-1] < 2.8
