"""Seeded synthetic workloads (inputs only; no walk arithmetic).

Each workload names an R-MAT graph (scale, edge factor, quadrant
probabilities, seed, weights) and a walk batch (starts, L, p, q, seed).  The
paper measures on real social graphs and on R-MAT graphs (Section 4.1); the
R-MAT graphs here stand in for both.  Starts are every vertex repeated r times
(walk k*n + v starts at v), the node2vec workload of r walks per vertex.
"""
from __future__ import annotations

import re
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    scale: int
    edge_factor: int
    a: float
    b: float
    c: float
    gseed: int
    weighted: bool
    p: float
    q: float
    r: int          # walks per vertex
    L: int          # moves per walk
    seed: int       # walk seed

    @property
    def n(self) -> int:
        return 1 << self.scale

    @property
    def walks(self) -> int:
        return self.r * self.n

    def rmat_args(self):
        return (self.scale, self.edge_factor, self.a, self.b, self.c, self.gseed)

    def starts(self, lo: int = 0, hi: int | None = None) -> np.ndarray:
        """Start ids of walks [lo, hi): walk w starts at w mod n."""
        hi = self.walks if hi is None else hi
        return (np.arange(lo, hi, dtype=np.uint64) % self.n).astype(np.uint32)

    def sample_walk_ids(self, count: int, seed: int = 0) -> np.ndarray:
        """A seeded uniform sample of walk ids (sorted, distinct)."""
        rng = np.random.default_rng(seed)
        count = min(count, self.walks)
        return np.sort(rng.choice(self.walks, size=count, replace=False)).astype(np.uint64)


RMAT_DEFAULT = (0.57, 0.19, 0.19)
RMAT_SKEW = (0.65, 0.15, 0.15)

# R-MAT scale 12, unweighted, p=0.5 q=2, r=10, L=80
C1 = Workload("rmat12-p0.5-q2-r10-L80", 12, 16, *RMAT_DEFAULT, 12, False, 0.5, 2.0, 10, 80, 1)
# R-MAT scale 20, weights uniform in [1,1000], p=1 q=0.5, r=10, L=80
C2 = Workload("rmat20w-p1-q0.5-r10-L80", 20, 16, *RMAT_DEFAULT, 20, True, 1.0, 0.5, 10, 80, 2)
# R-MAT scale 24 (a=.65, b=c=.15), unweighted, p=0.25 q=4, r=4, L=80
C3 = Workload("rmat24skew-p0.25-q4-r4-L80", 24, 16, *RMAT_SKEW, 24, False, 0.25, 4.0, 4, 80, 3)
# R-MAT scale 22 resident graph of the serving workload
C4 = Workload("rmat22-serving", 22, 16, *RMAT_DEFAULT, 22, False, 1.0, 1.0, 1, 80, 4)
# R-MAT scale 27, p=2 q=0.5, r=1, L=80, visit counts and checksum
C5 = Workload("rmat27-p2-q0.5-r1-L80-counts", 27, 16, *RMAT_DEFAULT, 27, False, 2.0, 0.5, 1, 80, 5)

ALL = {w.name: w for w in (C1, C2, C3, C4, C5)}


# The paper's synthetic families (Section 4.1), walked as in its measurements:
# one 80-move walk from every vertex.  Its |E| counts stored (directed) CSR
# entries: Table 1 lists ER-20 with 10.5M edges and maximum degree 29, Skew-1
# with 419.4M edges and maximum degree 159, which a symmetrized graph of
# edge_factor * 2^K generated edges matches with edge factors 5 and 50 (mean
# degrees 10 and 100), not 10 and 100.
PAPER_PQ = ((0.5, 2.0), (2.0, 0.5))


def _tag(x: float) -> str:
    return f"{x:g}"


def skew(S: float, p: float = 0.5, q: float = 2.0) -> Workload:
    """Skew-S: 2^22 vertices, mean degree 100, b = c = 1/4 and d = S * a."""
    a = 0.5 / (1.0 + S)
    return Workload(f"skew{_tag(S)}-p{_tag(p)}-q{_tag(q)}-r1-L80", 22, 50, a, 0.25, 0.25, 22, False, p, q, 1, 80, 6)


def wec(K: int, p: float = 0.5, q: float = 2.0) -> Workload:
    """WeC-K: 2^K vertices, 100 * 2^K entries, (a, b, c, d) = (.18, .25, .25, .32)."""
    return Workload(f"wec{K}-p{_tag(p)}-q{_tag(q)}-r1-L80", K, 50, 0.18, 0.25, 0.25, K, False, p, q, 1, 80, 7)


def er(K: int, p: float = 0.5, q: float = 2.0) -> Workload:
    """ER-K: 2^K vertices, mean degree 10, uniform quadrants."""
    return Workload(f"er{K}-p{_tag(p)}-q{_tag(q)}-r1-L80", K, 5, 0.25, 0.25, 0.25, K, False, p, q, 1, 80, 8)


def paper_family(name: str, p: float = 0.5, q: float = 2.0) -> Workload:
    """'skew<S>', 'wec<K>' or 'er<K>' (for example 'skew3', 'wec22', 'er26')."""
    m = re.fullmatch(r"(skew|wec|er)([0-9]+(?:\.[0-9]+)?)", name)
    if not m:
        raise ValueError(f"not a paper workload name: {name!r}")
    fam, x = m.group(1), m.group(2)
    if fam == "skew":
        return skew(float(x), p, q)
    if "." in x:
        raise ValueError(f"{fam} takes an integer scale: {name!r}")
    return (wec if fam == "wec" else er)(int(x), p, q)


# Table 1 of the paper (|E| and maximum degree of its generated graphs, made by
# another generator, so order-of-magnitude targets only).
PAPER_TABLE1 = {
    "er20": (10.5e6, 29), "er22": (41.9e6, 31), "er24": (167.8e6, 31), "er26": (671.1e6, 32),
    "er28": (2.7e9, 33), "er30": (10.7e9, 35),
    "wec20": (104.8e6, 1053), "wec22": (419.4e6, 1745), "wec26": (6.7e9, 2771),
    "skew1": (419.4e6, 159), "skew2": (419.4e6, 2098), "skew3": (419.4e6, 8420),
    "skew4": (419.2e6, 23594), "skew5": (418.3e6, 36914),
}

# FN-Base seconds on the paper's 12-machine cluster for all-vertex 80-step
# walks at p = 0.5, q = 2 (Section 4.6): other hardware, context only.
PAPER_FN_BASE_SECONDS = {"skew1.78": 314.5, "skew2": 369.3, "skew3": 811.1, "skew4": 1710.4, "skew5": 2913.4}


def philox_np(k0: int, k1: int, c0, c1, c2, c3):
    """Philox4x32-10 (Salmon et al., SC'11) over numpy arrays of counter words,
    for drawing inputs (request streams); returns four uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & 0xFFFFFFFF for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0, k1 = np.uint64(k0 & 0xFFFFFFFF), np.uint64(k1 & 0xFFFFFFFF)
    m32 = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(0xD2511F53) * c0
        p1 = np.uint64(0xCD9E8D57) * c2
        c0, c1, c2, c3 = (p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & m32, (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & m32
        k0 = (k0 + np.uint64(0x9E3779B9)) & m32
        k1 = (k1 + np.uint64(0xBB67AE85)) & m32
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


SERVING_PQ = (0.25, 0.5, 1.0, 2.0, 4.0)
SERVING_L = (20, 40, 80)


def serving_request(j: int, n: int, master: int = 4, size: int | None = None, max_log2: int = 20):
    """Request j of the serving stream, drawn from Philox with key = master and
    counters tagged 4: size floor(2^(max_log2 U)) in [1, 2^max_log2] (or `size`),
    L uniform over {20, 40, 80}, p and q uniform over {1/4, 1/2, 1, 2, 4}, starts
    uniform over [0, n), its own 63-bit seed and a uniform U for its arrival gap."""
    k0, k1 = master & 0xFFFFFFFF, master >> 32
    r = [int(x) for x in philox_np(k0, k1, j, 0, 0, 4)]
    if size is None:
        size = int(np.floor(2.0 ** (max_log2 * (r[0] / 2.0**32))))
        size = max(1, min(size, 1 << max_log2))
    L = SERVING_L[(r[1] * 3) >> 32]
    p = SERVING_PQ[(r[2] * 5) >> 32]
    q = SERVING_PQ[(r[3] * 5) >> 32]
    s = [int(x) for x in philox_np(k0, k1, j, 1, 0, 4)]
    seed = ((s[0] << 32) | s[1]) >> 1
    gap_u = (s[2] + 0.5) / 2.0**32
    i = np.arange(size, dtype=np.uint64)
    words = philox_np(k0, k1, j, 2, i >> np.uint64(2), 4)
    w = np.choose((i & np.uint64(3)).astype(np.int64), words).astype(np.uint64)
    starts = ((w * np.uint64(n)) >> np.uint64(32)).astype(np.uint32)
    return {"starts": starts, "L": L, "p": p, "q": q, "seed": seed, "gap_u": gap_u}


def serving_requests(count: int, n: int, first: int = 0, master: int = 4, max_log2: int = 20):
    """Requests first .. first+count-1 of the Philox-drawn serving stream."""
    return [serving_request(j, n, master, max_log2=max_log2) for j in range(first, first + count)]


def arrival_times(reqs, rate: float):
    """Poisson arrivals at `rate` requests per second: exponential gaps from each
    request's own uniform draw."""
    t, out = 0.0, []
    for r in reqs:
        t += -np.log(1.0 - r["gap_u"]) / rate
        out.append(t)
    return out


# FN-Approx speedup over FN-Base at the ends of the skew study (Section 4.6).
PAPER_FN_APPROX_SPEEDUP = {("skew1.78", 0.5, 2.0): 1.45, ("skew5", 0.5, 2.0): 17.2,
                           ("skew1.78", 2.0, 0.5): 1.41, ("skew5", 2.0, 0.5): 17.1}
