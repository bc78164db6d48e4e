"""CPU oracle for node2vec second-order walks (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()``, the CPU-baseline leg of
``bench.py`` and this package's own FN-Approx distance report
(``oracle/approx_distance.py``) import it.  It wraps ``oracle.c`` (plain C, built with
gcc by ``oracle/build.py``) and shares nothing with the GPU library.  See the
header of ``oracle.c`` for the definitions each function follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SENT = 0xFFFFFFFF

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    u32, u64, i32, dbl, vp = C.c_uint32, C.c_uint64, C.c_int, C.c_double, C.c_void_p
    lib.or_philox.argtypes = [u32, u32, vp, vp]
    lib.or_philox.restype = None
    lib.or_hi64.argtypes = [u64, u64]
    lib.or_hi64.restype = u64
    lib.or_rmat_thresholds.argtypes = [dbl, dbl, dbl, vp]
    lib.or_rmat_thresholds.restype = None
    lib.or_rmat_raw.argtypes = [u32, dbl, dbl, dbl, u64, u64, u64, vp, vp, i32]
    lib.or_rmat_raw.restype = None
    lib.or_pair_weight.argtypes = [u64, u32, u32]
    lib.or_pair_weight.restype = C.c_uint16
    lib.or_rmat_csr.argtypes = [u32, u32, dbl, dbl, dbl, u64, vp, vp, vp, u64, vp, i32]
    lib.or_rmat_csr.restype = i32
    lib.or_graph_new.argtypes = [vp, vp, vp, u32]
    lib.or_graph_new.restype = vp
    lib.or_graph_free.argtypes = [vp]
    lib.or_graph_free.restype = None
    lib.or_multipliers.argtypes = [dbl, dbl, vp]
    lib.or_multipliers.restype = i32
    lib.or_walk.argtypes = [vp, vp, vp, u64, u64, u32, dbl, dbl, u64, u32, u32, u32, vp, vp, vp, vp, i32]
    lib.or_walk.restype = i32
    lib.or_step_hist.argtypes = [vp, u32, u32, u32, u32, u64, dbl, dbl, u64, u32, u32, u32, vp]
    lib.or_step_hist.restype = i32
    lib.or_entry_hash.argtypes = [u64, u32, u32, u32]
    lib.or_entry_hash.restype = u64
    lib.or_walk_cost.argtypes = [vp, vp, vp, u64, u32, dbl, dbl, u64, u32, u32, u32, vp, vp, vp, i32]
    lib.or_walk_cost.restype = i32
    lib.or_step_cost.argtypes = [vp, u64, u32, u32, u32, u32, vp, u32, u32, u32, vp]
    lib.or_step_cost.restype = u64
    lib.or_walk_cost_classes.argtypes = [vp, vp, vp, u64, u32, dbl, dbl, u64, u32, u32, u32, vp, i32]
    lib.or_walk_cost_classes.restype = i32
    lib.or_memo_off_lines.argtypes = [u32]
    lib.or_memo_off_lines.restype = u64
    lib.or_memo_search_levels.argtypes = [u64]
    lib.or_memo_search_levels.restype = u64
    lib.or_memo_pair_lines.argtypes = [vp, u32, u32]
    lib.or_memo_pair_lines.restype = u64
    lib.or_memo_cold_lines.argtypes = [vp, i32, u32, u32]
    lib.or_memo_cold_lines.restype = u64
    lib.or_memo_warm_lines.argtypes = [vp, i32, u32, u32]
    lib.or_memo_warm_lines.restype = u64
    lib.or_memo_row_bytes.argtypes = [u64, i32]
    lib.or_memo_row_bytes.restype = u64
    lib.or_memo_pass_bytes.argtypes = [vp, i32, vp, u64, u32, u32, u32, i32, vp]
    lib.or_memo_pass_bytes.restype = i32
    lib.or_approx_bounds.argtypes = [u64, u64, vp, u32, u32, vp, vp, vp, vp]
    lib.or_approx_bounds.restype = None
    lib.or_approx_gap_below.argtypes = [u64, u64, vp, u32, u32, u32]
    lib.or_approx_gap_below.restype = i32
    lib.or_approx_applies.argtypes = [vp, u32, u32, vp, u32, u32]
    lib.or_approx_applies.restype = i32
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------
def philox(key, ctr):
    """Philox4x32-10 of one (key[2], ctr[4]) -> 4 words."""
    k = [int(x) & 0xFFFFFFFF for x in key]
    c = np.array([int(x) & 0xFFFFFFFF for x in ctr], dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().or_philox(k[0], k[1], _ptr(c), _ptr(out))
    return [int(x) for x in out]


def hi64(x: int, y: int) -> int:
    return int(_load().or_hi64(x, y))


def rmat_thresholds(a, b, c):
    T = np.zeros(3, dtype=np.uint64)
    _load().or_rmat_thresholds(a, b, c, _ptr(T))
    return [int(x) for x in T]


def rmat_raw(scale, a, b, c, gseed, e0, count, nthreads=None):
    """Raw R-MAT edges e0 .. e0+count-1 (before loop removal and symmetrisation)."""
    u = np.zeros(count, dtype=np.uint32)
    v = np.zeros(count, dtype=np.uint32)
    _load().or_rmat_raw(scale, a, b, c, gseed, e0, count, _ptr(u), _ptr(v),
                        nthreads or default_threads())
    return u, v


def pair_weight(gseed, x, y):
    return int(_load().or_pair_weight(gseed, x, y))


def multipliers(p, q):
    A = np.zeros(3, dtype=np.uint32)
    if _load().or_multipliers(p, q, _ptr(A)) != 0:
        raise ValueError("p and q must be in {0.25, 0.5, 1, 2, 4}")
    return [int(x) for x in A]


def entry_hash(seed, wid, col, x):
    return int(_load().or_entry_hash(seed, wid, col, x))


# --------------------------------------------------------------------------
# graphs
# --------------------------------------------------------------------------
class CSR:
    """A CSR graph held in numpy arrays (off u64[n+1], adj u32[m], wt u16[m] or None)."""

    def __init__(self, off, adj, wt=None):
        self.off = np.ascontiguousarray(off, dtype=np.uint64)
        self.adj = np.ascontiguousarray(adj, dtype=np.uint32)
        self.wt = None if wt is None else np.ascontiguousarray(wt, dtype=np.uint16)
        self.n = len(self.off) - 1
        self.m = int(self.off[-1])
        self._h = None

    @property
    def handle(self):
        if self._h is None:
            self._h = _load().or_graph_new(_ptr(self.off), _ptr(self.adj), _ptr(self.wt), self.n)
            if not self._h:
                raise MemoryError("oracle graph")
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.or_graph_free(self._h)
            self._h = None

    def degree(self):
        return np.diff(self.off.astype(np.int64))

    def row(self, v):
        return self.adj[int(self.off[v]):int(self.off[v + 1])]

    @staticmethod
    def from_edges(n, edges, weights=None):
        """Symmetric CSR from undirected edge pairs (dedup, loops dropped).

        weights: optional dict {(min,max): w}."""
        rows = [set() for _ in range(n)]
        for a, b in edges:
            if a == b:
                continue
            rows[a].add(b)
            rows[b].add(a)
        off = np.zeros(n + 1, dtype=np.uint64)
        adj = []
        wt = [] if weights is not None else None
        for v in range(n):
            r = sorted(rows[v])
            adj.extend(r)
            if wt is not None:
                wt.extend(weights[(min(v, x), max(v, x))] for x in r)
            off[v + 1] = off[v] + len(r)
        return CSR(off, np.array(adj, dtype=np.uint32),
                   None if wt is None else np.array(wt, dtype=np.uint16))


def rmat_csr(scale, edge_factor, a, b, c, gseed, weighted=False, nthreads=None):
    """CSR of the symmetrised, de-duplicated, loop-free R-MAT graph."""
    n = 1 << scale
    cap = 2 * (edge_factor << scale)
    off = np.zeros(n + 1, dtype=np.uint64)
    adj = np.zeros(cap, dtype=np.uint32)
    wt = np.zeros(cap, dtype=np.uint16) if weighted else None
    m = np.zeros(1, dtype=np.uint64)
    rc = _load().or_rmat_csr(scale, edge_factor, a, b, c, gseed, _ptr(off), _ptr(adj),
                             _ptr(wt), cap, _ptr(m), nthreads or default_threads())
    if rc != 0:
        raise RuntimeError(f"or_rmat_csr failed ({rc})")
    mm = int(m[0])
    adj = adj[:mm].copy()
    if wt is not None:
        wt = wt[:mm].copy()
    return CSR(off, adj, wt)


# --------------------------------------------------------------------------
# walks
# --------------------------------------------------------------------------
D_RULE = 1024
A_CAP = 1024


def walk(g: CSR, starts, L, p, q, seed, walk_base=0, wids=None, d_rule=D_RULE, a_cap=A_CAP,
         want_out=True, want_counts=False, nthreads=None, approx_t=0):
    """Runs the walks; returns dict(out, cnt, checksum, transitions).  approx_t > 0
    applies FN-Approx (Section 3.4) with threshold 1/approx_t."""
    starts = np.ascontiguousarray(starts, dtype=np.uint32)
    count = len(starts)
    wid_arr = None if wids is None else np.ascontiguousarray(wids, dtype=np.uint64)
    out = np.zeros((count, L + 1), dtype=np.uint32) if want_out else None
    cnt = np.zeros(g.n, dtype=np.uint32) if want_counts else None
    cs = np.zeros(1, dtype=np.uint64)
    tr = np.zeros(1, dtype=np.uint64)
    rc = _load().or_walk(g.handle, _ptr(starts), _ptr(wid_arr), walk_base, count, L, p, q, seed,
                         d_rule, a_cap, approx_t, _ptr(out), _ptr(cnt), _ptr(cs), _ptr(tr),
                         nthreads or default_threads())
    if rc != 0:
        raise ValueError("bad walk arguments (p, q or a start id)")
    return {"out": out, "cnt": cnt, "checksum": int(cs[0]), "transitions": int(tr[0])}


def step_hist(g: CSR, t, v, s, draws, p, q, seed, wid0=0, d_rule=D_RULE, a_cap=A_CAP, approx_t=0):
    """Counts of each neighbour index of v chosen over `draws` single moves at (t, v, s)."""
    d = int(g.off[v + 1] - g.off[v])
    hist = np.zeros(d, dtype=np.uint64)
    rc = _load().or_step_hist(g.handle, t, v, s, wid0, draws, p, q, seed, d_rule, a_cap, approx_t, _ptr(hist))
    if rc != 0:
        raise ValueError("bad step arguments")
    return hist


def walk_cost(g: CSR, starts, wids, L, p, q, seed, d_rule=D_RULE, a_cap=A_CAP, nthreads=None, approx_t=0):
    """(algorithmic bytes, moves, moves at vertices above d_rule) summed over the walks."""
    starts = np.ascontiguousarray(starts, dtype=np.uint32)
    wids = np.ascontiguousarray(wids, dtype=np.uint64)
    b = np.zeros(1, dtype=np.uint64)
    s = np.zeros(1, dtype=np.uint64)
    h = np.zeros(1, dtype=np.uint64)
    rc = _load().or_walk_cost(g.handle, _ptr(starts), _ptr(wids), len(starts), L, p, q, seed,
                              d_rule, a_cap, approx_t, _ptr(b), _ptr(s), _ptr(h), nthreads or default_threads())
    if rc != 0:
        raise ValueError("bad cost arguments")
    return int(b[0]), int(s[0]), int(h[0])


def step_cost(g: CSR, seed, wid, s, t, v, p, q, d_rule=D_RULE, a_cap=A_CAP, approx_t=0):
    """Isolated algorithmic bytes of one move (walk wid, step s, at v after t) and its result."""
    A = np.array(multipliers(p, q), dtype=np.uint32)
    nxt = np.zeros(1, dtype=np.uint32)
    b = _load().or_step_cost(g.handle, seed, wid, s, t, v, _ptr(A), d_rule, a_cap, approx_t, _ptr(nxt))
    return int(b), int(nxt[0])


def walk_cost_classes(g: CSR, starts, wids, L, p, q, seed, d_rule=D_RULE, a_cap=A_CAP, nthreads=None, approx_t=0):
    """Isolated algorithmic bytes split by class: (bytes, moves) of second-order moves at
    vertices above d_rule, then (bytes, moves) of every other move."""
    starts = np.ascontiguousarray(starts, dtype=np.uint32)
    wids = np.ascontiguousarray(wids, dtype=np.uint64)
    cls = np.zeros(4, dtype=np.uint64)
    rc = _load().or_walk_cost_classes(g.handle, _ptr(starts), _ptr(wids), len(starts), L, p, q, seed,
                                      d_rule, a_cap, approx_t, _ptr(cls), nthreads or default_threads())
    if rc != 0:
        raise ValueError("bad cost arguments")
    return tuple(int(x) for x in cls)


# memo-aware bytes model of a pass (see oracle.c: or_memo_pass_bytes)
MEMO_MAX_DEG = 4161536


def memo_off_lines(v):
    return int(_load().or_memo_off_lines(v))


def memo_search_levels(d):
    return int(_load().or_memo_search_levels(d))


def memo_pair_lines(off, a, b):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    return int(_load().or_memo_pair_lines(_ptr(off), a, b))


def memo_cold_lines(off, t, v, weighted=False):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    return int(_load().or_memo_cold_lines(_ptr(off), int(weighted), t, v))


def memo_warm_lines(off, t, v, weighted=False):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    return int(_load().or_memo_warm_lines(_ptr(off), int(weighted), t, v))


def memo_row_bytes(d, weighted=False):
    """Bytes of one pair-summary row of a vertex of degree d (or_memo_row_bytes)."""
    return int(_load().or_memo_row_bytes(int(d), int(weighted)))


def memo_pass_bytes(off, out, L, d_rule=D_RULE, memo_min=None, memo=True, weighted=False):
    """Memo-aware bytes of a pass given by its walk matrix: dict(hub_bytes, hub_moves,
    other_moves, intersections, warm_moves)."""
    off = np.ascontiguousarray(off, dtype=np.uint64)
    out = np.ascontiguousarray(out, dtype=np.uint32)
    res = np.zeros(5, dtype=np.uint64)
    mm = d_rule + 1 if memo_min is None else memo_min
    rc = _load().or_memo_pass_bytes(_ptr(off), int(weighted), _ptr(out), out.shape[0], L, d_rule, mm, int(memo),
                                    _ptr(res))
    if rc != 0:
        raise MemoryError("or_memo_pass_bytes")
    return dict(zip(["hub_bytes", "hub_moves", "other_moves", "intersections", "warm_moves"],
                    (int(x) for x in res)))


def approx_bounds(du, dv, p, q, wlo=1, whi=1):
    """FN-Approx bounds (Section 3.4, Eqs. 2 and 3) on the probability of a
    move v -> x, x != u, after u -> v: (LB, UB) as Fractions."""
    from fractions import Fraction
    A = np.array(multipliers(p, q), dtype=np.uint32)
    out = [np.zeros(1, dtype=np.uint64) for _ in range(4)]
    _load().or_approx_bounds(du, dv, _ptr(A), wlo, whi, *[_ptr(o) for o in out])
    ln, ld, un, ud = (int(o[0]) for o in out)
    return Fraction(ln, ld), Fraction(un, ud)


def approx_gap_below(du, dv, p, q, approx_t, wlo=1, whi=1):
    """UB - LB < 1/approx_t, as the oracle decides it (128-bit cross-multiplication)."""
    A = np.array(multipliers(p, q), dtype=np.uint32)
    return bool(_load().or_approx_gap_below(du, dv, _ptr(A), wlo, whi, approx_t))


def approx_applies(g: CSR, t, v, p, q, approx_t, d_rule=D_RULE):
    """Whether FN-Approx draws the move at v after t from the static weights."""
    A = np.array(multipliers(p, q), dtype=np.uint32)
    return bool(_load().or_approx_applies(g.handle, t, v, _ptr(A), d_rule, approx_t))


def visit_profile(g: CSR, cnt, width, nbuckets):
    """Vertices and summed visits per equi-width degree bucket (Section 3.3,
    the frequency-versus-degree figure): bucket 0 is degree 0, bucket k >= 1
    degrees in ((k-1) width, k width], the last bucket also every larger degree."""
    deg = np.diff(g.off.astype(np.int64))
    b = np.minimum(-(-deg // width), nbuckets - 1)
    verts = np.bincount(b, minlength=nbuckets).astype(np.int64)
    visits = np.zeros(nbuckets, dtype=np.int64)
    np.add.at(visits, b, np.asarray(cnt, dtype=np.int64))
    return verts, visits


def checksum_of(out, seed, walk_ids):
    """Visit counts and checksum of a walk matrix, entry by entry (slow; small inputs)."""
    total = 0
    for i, row in enumerate(out):
        wid = int(walk_ids[i]) & 0xFFFFFFFF
        for col, x in enumerate(row):
            if int(x) == SENT:
                break
            total = (total + entry_hash(seed, wid, col, int(x))) & 0xFFFFFFFFFFFFFFFF
    return total
