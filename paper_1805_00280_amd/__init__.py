"""MI355X node2vec walk engine: Python binding of the C ABI in include/n2v.h.

The binding only marshals arguments: every step of graph generation, graph
preparation and walking runs in the HIP kernels of libn2v.so.  PyTorch is used
for device memory and streams.  Importing works without a GPU; every call that
reaches the library fails loudly when libn2v.so is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# N2V_LIBRARY selects another build of the same library (e.g. a variant under test)
LIB_PATH = os.environ.get("N2V_LIBRARY") or os.path.join(_HERE, "libn2v.so")
SENT = 0xFFFFFFFF

N2V_OK, N2V_PENDING = 0, 1
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EGRAPH", -4: "EDEVICE", -5: "EAGAIN", -6: "ETOOBIG", -7: "ENOTFOUND"}
MODE_AUTO, MODE_PLAIN, MODE_PERSISTENT = 0, 1, 2
OUT_WALKS, OUT_COUNTS = 1, 2

# Every symbol include/n2v.h declares.
EXPORTS = [
    "n2v_last_error", "n2v_abi_version",
    "n2v_rmat_workspace", "n2v_rmat_generate",
    "n2v_graph_opts_default", "n2v_graph_workspace", "n2v_graph_create", "n2v_graph_destroy",
    "n2v_graph_info", "n2v_graph_check", "n2v_graph_memo_bytes", "n2v_graph_set_memo",
    "n2v_graph_memo_plan", "n2v_graph_set_memo_min", "n2v_graph_memo_clear",
    "n2v_exec_opts_default", "n2v_walk", "n2v_walk_workspace", "n2v_walk_ex", "n2v_walk_approx", "n2v_walk_static",
    "n2v_visit_profile",
    "n2v_sgns_workspace", "n2v_sgns_negatives", "n2v_sgns_step",
    "n2v_autotune_workspace", "n2v_autotune",
    "n2v_server_opts_default", "n2v_server_create", "n2v_server_destroy", "n2v_submit", "n2v_poll",
    "n2v_release", "n2v_server_stats",
]


class N2VError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class RmatParams(C.Structure):
    _fields_ = [("scale", C.c_uint32), ("edge_factor", C.c_uint32), ("a", C.c_double), ("b", C.c_double),
                ("c", C.c_double), ("seed", C.c_uint64), ("weighted", C.c_int)]


class GraphOpts(C.Structure):
    _fields_ = [("d_rule", C.c_uint32), ("a_cap", C.c_uint32), ("validate", C.c_int)]


class ExecOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("t_wave", C.c_uint32), ("t_sparse", C.c_uint32),
                ("sparse_ratio", C.c_uint32), ("waves_per_cu", C.c_uint32), ("block", C.c_uint32),
                ("memo", C.c_uint32), ("t_wg", C.c_uint32),
                ("search_ratio", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("max_queue", C.c_uint32), ("chunk_walks", C.c_uint32), ("max_inflight", C.c_uint32),
                ("tick_walks", C.c_uint32)]


class Request(C.Structure):
    _fields_ = [("host_starts", C.c_void_p), ("n_starts", C.c_uint32), ("L", C.c_uint32), ("p", C.c_float),
                ("q", C.c_float), ("seed", C.c_uint64), ("approx_t", C.c_uint32)]


class SgnsParams(C.Structure):
    _fields_ = [("dim", C.c_uint32), ("window", C.c_uint32), ("negatives", C.c_uint32), ("neg_weight", C.c_float),
                ("lr", C.c_float), ("seed", C.c_uint64), ("step", C.c_uint32)]


class Result(C.Structure):
    _fields_ = [("d_out", C.c_void_p), ("n_starts", C.c_uint32), ("L", C.c_uint32), ("submit_ns", C.c_uint64),
                ("start_ns", C.c_uint64), ("done_ns", C.c_uint64)]


ABI_VERSION = 7  # layout of the option structs and sketch rows, entry points
_lib = None


def lib():
    """The loaded libn2v.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libn2v.so not found at {LIB_PATH}: build it with "
                           f"`python -m paper_1805_00280_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, u32, u64, i32, f32, sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int, C.c_float, C.c_size_t
    P = C.POINTER
    sig = {
        "n2v_last_error": ([], C.c_char_p),
        "n2v_abi_version": ([], i32),
        "n2v_rmat_workspace": ([P(RmatParams), P(sz), P(u64)], i32),
        "n2v_rmat_generate": ([P(RmatParams), vp, sz, vp, vp, vp, P(u64), vp], i32),
        "n2v_graph_opts_default": ([P(GraphOpts)], None),
        "n2v_graph_workspace": ([u32, u64, i32, P(sz)], i32),
        "n2v_graph_create": ([vp, vp, vp, u32, u64, P(GraphOpts), vp, sz, vp, P(vp)], i32),
        "n2v_graph_destroy": ([vp], i32),
        "n2v_graph_info": ([vp, P(u32), P(u64), P(u32), P(u32), P(i32)], i32),
        "n2v_graph_check": ([vp, vp], i32),
        "n2v_graph_memo_bytes": ([vp, P(sz)], i32),
        "n2v_graph_set_memo": ([vp, vp, sz], i32),
        "n2v_graph_memo_plan": ([vp, sz, P(u32), P(sz)], i32),
        "n2v_graph_set_memo_min": ([vp, vp, sz, u32], i32),
        "n2v_graph_memo_clear": ([vp, vp], i32),
        "n2v_exec_opts_default": ([vp, P(ExecOpts)], None),
        "n2v_walk": ([vp, vp, u32, u32, f32, f32, u64, vp, vp], i32),
        "n2v_walk_workspace": ([vp, u32, u32, P(ExecOpts), P(sz)], i32),
        "n2v_walk_ex": ([vp, vp, u32, u64, u32, f32, f32, u64, P(ExecOpts), i32, vp, vp, vp, vp, sz, vp], i32),
        "n2v_walk_approx": ([vp, vp, u32, u64, u32, f32, f32, u64, u32, P(ExecOpts), i32, vp, vp, vp, vp, sz, vp],
                            i32),
        "n2v_walk_static": ([vp, vp, u32, u64, u32, f32, f32, u64, u32, P(ExecOpts), i32, vp, vp, vp, vp], i32),
        "n2v_visit_profile": ([vp, vp, u32, u32, vp, vp, vp], i32),
        "n2v_sgns_workspace": ([u32, u32, u32, u32, P(sz)], i32),
        "n2v_sgns_negatives": ([vp, u32, u64, u64, u32, u32, u32, vp, vp], i32),
        "n2v_sgns_step": ([P(SgnsParams), vp, u32, u32, u64, vp, u32, vp, vp, vp, sz, vp, vp], i32),
        "n2v_autotune_workspace": ([vp, u32, u32, P(sz)], i32),
        "n2v_autotune": ([vp, u32, u32, f32, f32, vp, sz, vp, P(ExecOpts), P(C.c_double)], i32),
        "n2v_server_opts_default": ([P(ServerOpts)], None),
        "n2v_server_create": ([vp, vp, sz, P(ServerOpts), vp, P(vp)], i32),
        "n2v_server_destroy": ([vp], i32),
        "n2v_submit": ([vp, P(Request), P(u64)], i32),
        "n2v_poll": ([vp, u64, P(Result)], i32),
        "n2v_release": ([vp, u64], i32),
        "n2v_server_stats": ([vp, P(u32), P(u32), P(u32)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    if L.n2v_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH}: ABI version {L.n2v_abi_version()}, this binding expects {ABI_VERSION}; "
                           "rebuild the library")
    _lib = L
    return L


def check(rc, what=""):
    if rc < 0:
        msg = lib().n2v_last_error().decode(errors="replace")
        raise N2VError(rc, f"{what}: {msg}" if what else msg)
    return rc


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _alloc(nbytes, device):
    """Device bytes (256-byte aligned by the caching allocator)."""
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def exec_opts(graph=None, **kw):
    o = ExecOpts()
    lib().n2v_exec_opts_default(graph._h if graph is not None else None, C.byref(o))
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, int(v))
    return o


# --------------------------------------------------------------------------
class Graph:
    """A graph resident on the GPU (CSR plus derived arrays)."""

    def __init__(self, off, adj, wt=None, n=None, d_rule=1024, a_cap=1024, validate=1, stream=None):
        torch = _torch()
        self.off, self.adj, self.wt = off, adj, wt
        self.n = int(n if n is not None else off.numel() - 1)
        self.m = int(adj.numel())
        self.device = off.device
        ws = C.c_size_t()
        check(lib().n2v_graph_workspace(self.n, self.m, int(wt is not None), C.byref(ws)), "n2v_graph_workspace")
        self.ws = _alloc(ws.value, self.device)
        o = GraphOpts(d_rule, a_cap, validate)
        h = C.c_void_p()
        check(lib().n2v_graph_create(_ptr(off), _ptr(adj), _ptr(wt), self.n, self.m, C.byref(o), _ptr(self.ws),
                                     self.ws.numel(), _stream(stream), C.byref(h)), "n2v_graph_create")
        self._h = h
        self.d_rule, self.a_cap = d_rule, a_cap
        self.weighted = wt is not None
        self.memo = None
        self.memo_min_degree = None
        del torch

    @staticmethod
    def generate_rmat(scale, edge_factor, a, b, c, seed, weighted=False, device="cuda", stream=None):
        """On-device R-MAT CSR: returns (off int64[n+1], adj int32[m], wt int16[m] or None)."""
        torch = _torch()
        prm = RmatParams(scale, edge_factor, a, b, c, seed, int(weighted))
        ws = C.c_size_t()
        mmax = C.c_uint64()
        check(lib().n2v_rmat_workspace(C.byref(prm), C.byref(ws), C.byref(mmax)), "n2v_rmat_workspace")
        n = 1 << scale
        off = torch.empty(n + 1, dtype=torch.int64, device=device)
        adj = torch.empty(mmax.value, dtype=torch.int32, device=device)
        wt = torch.empty(mmax.value, dtype=torch.int16, device=device) if weighted else None
        work = _alloc(ws.value, device)
        m = C.c_uint64()
        check(lib().n2v_rmat_generate(C.byref(prm), _ptr(work), work.numel(), _ptr(off), _ptr(adj), _ptr(wt),
                                      C.byref(m), _stream(stream)), "n2v_rmat_generate")
        del work
        mm = m.value
        adj = adj[:mm].clone()
        if wt is not None:
            wt = wt[:mm].clone()
        return off, adj, wt

    @classmethod
    def from_rmat(cls, scale, edge_factor, a, b, c, seed, weighted=False, d_rule=1024, a_cap=1024,
                  device="cuda", stream=None, validate=1):
        off, adj, wt = cls.generate_rmat(scale, edge_factor, a, b, c, seed, weighted, device, stream)
        return cls(off, adj, wt, n=1 << scale, d_rule=d_rule, a_cap=a_cap, validate=validate, stream=stream)

    @classmethod
    def from_numpy(cls, off, adj, wt=None, device="cuda", **kw):
        torch = _torch()
        t_off = torch.from_numpy(np.ascontiguousarray(off, dtype=np.uint64).view(np.int64)).to(device)
        t_adj = torch.from_numpy(np.ascontiguousarray(adj, dtype=np.uint32).view(np.int32)).to(device)
        t_wt = None
        if wt is not None:
            t_wt = torch.from_numpy(np.ascontiguousarray(wt, dtype=np.uint16).view(np.int16)).to(device)
        return cls(t_off, t_adj, t_wt, n=len(off) - 1, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().n2v_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n, m, d, a, w = C.c_uint32(), C.c_uint64(), C.c_uint32(), C.c_uint32(), C.c_int()
        check(lib().n2v_graph_info(self._h, C.byref(n), C.byref(m), C.byref(d), C.byref(a), C.byref(w)))
        return {"n": n.value, "m": m.value, "d_rule": d.value, "a_cap": a.value, "weighted": bool(w.value)}

    def attach_memo(self, budget=None):
        """Allocates and attaches pair-sketch memory (unweighted graphs); returns its bytes.  With a
        byte budget, only rows of the highest-degree vertices that fit keep sketches (0 if none)."""
        # the previous memory stays referenced until the library has switched
        # to the new one (a refused attach leaves the graph on the old memory)
        if budget is None:
            b = C.c_size_t()
            check(lib().n2v_graph_memo_bytes(self._h, C.byref(b)), "n2v_graph_memo_bytes")
            if b.value == 0:
                return 0
            mem = _alloc(b.value, self.device)
            check(lib().n2v_graph_set_memo(self._h, _ptr(mem), mem.numel()), "n2v_graph_set_memo")
            self.memo = mem
            self.memo_min_degree = self.d_rule + 1
            return b.value
        dmin, b = C.c_uint32(), C.c_size_t()
        check(lib().n2v_graph_memo_plan(self._h, int(budget), C.byref(dmin), C.byref(b)), "n2v_graph_memo_plan")
        if b.value == 0:
            return 0
        mem = _alloc(b.value, self.device)
        check(lib().n2v_graph_set_memo_min(self._h, _ptr(mem), mem.numel(), dmin.value), "n2v_graph_set_memo_min")
        self.memo = mem
        self.memo_min_degree = dmin.value
        return b.value

    def memo_clear(self, stream=None):
        """Enqueues the clearing of the pair sketches: the next walk pass starts cold."""
        check(lib().n2v_graph_memo_clear(self._h, _stream(stream)), "n2v_graph_memo_clear")

    def detach_memo(self):
        check(lib().n2v_graph_set_memo(self._h, None, 0), "n2v_graph_set_memo")
        self.memo = None
        self.memo_min_degree = None

    def check_starts(self, stream=None):
        check(lib().n2v_graph_check(self._h, _stream(stream)), "n2v_graph_check")

    # ---------------------------------------------------------------- walks
    def walk_workspace(self, n_starts, L, opts):
        ws = C.c_size_t()
        check(lib().n2v_walk_workspace(self._h, n_starts, L, C.byref(opts), C.byref(ws)), "n2v_walk_workspace")
        return ws.value

    def _walk_call(self, starts, n, walk_base, L, p, q, seed, approx_t, o, outputs, out, cnt, checksum, ws, need,
                   stream):
        wsp, wsn = (_ptr(ws), ws.numel()) if need else (None, 0)
        if approx_t:
            check(lib().n2v_walk_approx(self._h, _ptr(starts), n, walk_base, L, p, q, seed, approx_t, C.byref(o),
                                        outputs, _ptr(out), _ptr(cnt), _ptr(checksum), wsp, wsn, _stream(stream)),
                  "n2v_walk_approx")
        else:
            check(lib().n2v_walk_ex(self._h, _ptr(starts), n, walk_base, L, p, q, seed, C.byref(o), outputs,
                                    _ptr(out), _ptr(cnt), _ptr(checksum), wsp, wsn, _stream(stream)), "n2v_walk_ex")

    def walk(self, starts, L, p, q, seed, walk_base=0, out=None, opts=None, stream=None, ws=None, approx_t=0, **kw):
        """Walk matrix (int32 view of uint32), n_starts x (L+1).  approx_t > 0
        applies FN-Approx with threshold 1/approx_t (n2v_walk_approx)."""
        torch = _torch()
        n = int(starts.numel())
        if out is None:
            out = torch.empty((n, L + 1), dtype=torch.int32, device=self.device)
        o = opts if opts is not None else exec_opts(self, **kw)
        need = self.walk_workspace(n, L, o)
        if need and ws is None:
            ws = _alloc(need, self.device)
        self._walk_call(starts, n, walk_base, L, p, q, seed, approx_t, o, OUT_WALKS, out, None, None, ws, need,
                        stream)
        return out

    def walk_static(self, starts, L, p, q, seed, walk_base=0, out=None, opts=None, stream=None, approx_t=0):
        """Plain form in the library's static scratch (n2v_walk_static): allocates nothing
        beyond `out` when it is not given."""
        torch = _torch()
        n = int(starts.numel())
        if out is None:
            out = torch.empty((n, L + 1), dtype=torch.int32, device=self.device)
        o = opts if opts is not None else exec_opts(self)
        check(lib().n2v_walk_static(self._h, _ptr(starts), n, walk_base, L, p, q, seed, approx_t, C.byref(o),
                                    OUT_WALKS, _ptr(out), None, None, _stream(stream)), "n2v_walk_static")
        return out

    def walk_simple(self, starts, L, p, q, seed, out=None, stream=None):
        torch = _torch()
        n = int(starts.numel())
        if out is None:
            out = torch.empty((n, L + 1), dtype=torch.int32, device=self.device)
        check(lib().n2v_walk(self._h, _ptr(starts), n, L, p, q, seed, _ptr(out), _stream(stream)), "n2v_walk")
        return out

    def walk_counts(self, starts, L, p, q, seed, cnt, checksum, walk_base=0, out=None, opts=None, stream=None,
                    ws=None, approx_t=0, **kw):
        """Adds visit counts into cnt (int32[n]) and the checksum into checksum (int64[1])."""
        n = int(starts.numel())
        o = opts if opts is not None else exec_opts(self, **kw)
        need = self.walk_workspace(n, L, o)
        if need and ws is None:
            ws = _alloc(need, self.device)
        outputs = OUT_COUNTS | (OUT_WALKS if out is not None else 0)
        self._walk_call(starts, n, walk_base, L, p, q, seed, approx_t, o, outputs, out, cnt, checksum, ws, need,
                        stream)

    def visit_profile(self, cnt, width, nbuckets, stream=None):
        """(vertices, visits) per degree bucket (int64 tensors of nbuckets): bucket 0 is
        degree 0, bucket k degrees in ((k-1) width, k width], the last also all larger."""
        torch = _torch()
        verts = torch.empty(nbuckets, dtype=torch.int64, device=self.device)
        visits = torch.empty(nbuckets, dtype=torch.int64, device=self.device)
        check(lib().n2v_visit_profile(self._h, _ptr(cnt), width, nbuckets, _ptr(verts), _ptr(visits),
                                      _stream(stream)), "n2v_visit_profile")
        return verts, visits

    def autotune(self, n_walks, L, p, q, stream=None):
        ws = C.c_size_t()
        check(lib().n2v_autotune_workspace(self._h, n_walks, L, C.byref(ws)), "n2v_autotune_workspace")
        work = _alloc(ws.value, self.device)
        best = ExecOpts()
        ms = C.c_double()
        check(lib().n2v_autotune(self._h, n_walks, L, p, q, _ptr(work), work.numel(), _stream(stream),
                                 C.byref(best), C.byref(ms)), "n2v_autotune")
        return best, ms.value


# --------------------------------------------------------------------------
class SkipGram:
    """Skip-gram with negative sampling over walks (n2v_sgns_step): embedding tables
    win and wout (n x 128 fp32, device) trained in steps over batches of walk rows."""

    DIM = 128

    def __init__(self, n, win, wout, cum, window=10, negatives=64, neg_weight=None, lr=0.025, seed=1,
                 max_walks=1 << 16, device="cuda"):
        torch = _torch()
        self.n, self.win, self.wout, self.device = n, win, wout, device
        self.cum = cum  # device u64 (int64 tensor) cumulative noise weights, n + 1
        k = 5 * 2 * window  # word2vec's 5 negatives per (center, context) pair, spread over the shared ones
        self.prm = SgnsParams(self.DIM, window, negatives, neg_weight if neg_weight is not None else k / negatives,
                              lr, seed, 0)
        ws = C.c_size_t()
        check(lib().n2v_sgns_workspace(n, self.DIM, max_walks, negatives, C.byref(ws)), "n2v_sgns_workspace")
        self.ws = torch.zeros(max(ws.value, 256), dtype=torch.uint8, device=device)
        self.max_walks = max_walks
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)

    def step(self, walks, walk_base=0, step=None, stream=None):
        """One SGD step over walk rows (int32 tensor view of uint32, n_walks x row_len)."""
        n_walks, row_len = int(walks.shape[0]), int(walks.shape[1])
        if n_walks > self.max_walks:
            raise ValueError(f"batch of {n_walks} walks exceeds the workspace's {self.max_walks}")
        if step is not None:
            self.prm.step = step
        check(lib().n2v_sgns_step(C.byref(self.prm), _ptr(walks), n_walks, row_len, walk_base, _ptr(self.cum), self.n,
                                  _ptr(self.win), _ptr(self.wout), _ptr(self.ws), self.ws.numel(), _ptr(self.loss),
                                  _stream(stream)), "n2v_sgns_step")
        self.prm.step += 1

    def negatives(self, n_walks, walk_base=0, step=0, stream=None):
        torch = _torch()
        out = torch.empty((n_walks, self.prm.negatives), dtype=torch.int32, device=self.device)
        check(lib().n2v_sgns_negatives(_ptr(self.cum), self.n, self.prm.seed, walk_base, step, n_walks,
                                       self.prm.negatives, _ptr(out), _stream(stream)), "n2v_sgns_negatives")
        return out


# --------------------------------------------------------------------------
@dataclass
class Done:
    out: object       # torch int32 tensor view of the device result (valid until release)
    submit_ns: int
    start_ns: int
    done_ns: int


class Server:
    """Continuous-batching walk server over a resident graph (see n2v.h)."""

    def __init__(self, graph: Graph, pool_bytes, chunk_walks=None, max_inflight=None, max_queue=None, stream=None,
                 tick_walks=None):
        torch = _torch()
        self.graph = graph
        self.pool = _alloc(pool_bytes, graph.device)
        o = ServerOpts()
        lib().n2v_server_opts_default(C.byref(o))
        if chunk_walks:
            o.chunk_walks = chunk_walks
        if max_inflight:
            o.max_inflight = max_inflight
        if max_queue:
            o.max_queue = max_queue
        if tick_walks:
            o.tick_walks = tick_walks
        self.stream = stream if stream is not None else torch.cuda.Stream(graph.device)
        h = C.c_void_p()
        check(lib().n2v_server_create(graph._h, _ptr(self.pool), self.pool.numel(), C.byref(o),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)), "n2v_server_create")
        self._h = h
        self._keep = {}

    def submit(self, starts_np, L, p, q, seed, approx_t=0):
        starts_np = np.ascontiguousarray(starts_np, dtype=np.uint32)
        r = Request(starts_np.ctypes.data, len(starts_np), L, p, q, seed, approx_t)
        t = C.c_uint64()
        rc = lib().n2v_submit(self._h, C.byref(r), C.byref(t))
        check(rc, "n2v_submit")
        return t.value

    def poll(self, ticket):
        res = Result()
        rc = lib().n2v_poll(self._h, ticket, C.byref(res))
        if rc == N2V_PENDING:
            return None
        check(rc, "n2v_poll")
        return res

    def result_tensor(self, res):
        """Copy of a completed result as a host numpy uint32 array."""
        torch = _torch()
        n = res.n_starts * (res.L + 1)
        buf = torch.empty(n, dtype=torch.int32, device=self.graph.device)
        _copy_d2d(buf, res.d_out, n * 4, self.stream)
        self.stream.synchronize()
        return buf.cpu().numpy().view(np.uint32).reshape(res.n_starts, res.L + 1)

    def release(self, ticket):
        check(lib().n2v_release(self._h, ticket), "n2v_release")

    def stats(self):
        a, b, c = C.c_uint32(), C.c_uint32(), C.c_uint32()
        check(lib().n2v_server_stats(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "_h", None):
            lib().n2v_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _copy_d2d(dst_tensor, src_ptr, nbytes, stream):
    """Device-to-device copy from a raw pointer through the HIP runtime torch already loaded."""
    hip = _hip_runtime()
    rc = hip.hipMemcpyAsync(C.c_void_p(dst_tensor.data_ptr()), C.c_void_p(src_ptr), C.c_size_t(nbytes), 3,
                            C.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        # the runtime torch already loaded (same soname), never a second copy
        _hip = C.CDLL("libamdhip64.so.7")
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
    return _hip


def as_u32(t):
    """Host numpy uint32 view of an int32 torch tensor."""
    return t.cpu().numpy().view(np.uint32)
