"""Seeded synthetic workloads (inputs only; no walk arithmetic).

Each workload names an R-MAT graph (scale, edge factor, quadrant
probabilities, seed, weights) and a walk batch (starts, L, p, q, seed).  The
paper measures on real social graphs and on R-MAT graphs (Section 4.1); the
R-MAT graphs here stand in for both.  Starts are every vertex repeated r times
(walk k*n + v starts at v), the node2vec workload of r walks per vertex.
"""
from __future__ import annotations

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


def serving_requests(count: int, n: int, seed: int = 4, max_log2: int = 20):
    """Request stream of the serving workload: sizes log-uniform in [1, 2^max_log2],
    L uniform in {20, 40, 80}, p and q uniform over {0.25, 0.5, 1, 2, 4}, starts
    uniform over the vertices, one seed per request."""
    rng = np.random.default_rng(seed)
    pq = np.array([0.25, 0.5, 1.0, 2.0, 4.0])
    out = []
    for j in range(count):
        size = int(np.floor(2.0 ** (max_log2 * rng.random())))
        size = max(1, min(size, 1 << max_log2))
        out.append({
            "starts": rng.integers(0, n, size=size, dtype=np.uint64).astype(np.uint32),
            "L": int(rng.choice([20, 40, 80])),
            "p": float(rng.choice(pq)),
            "q": float(rng.choice(pq)),
            "seed": int(rng.integers(0, 2**63)),
        })
    return out
