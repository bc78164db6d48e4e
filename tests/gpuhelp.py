"""Helpers shared by the GPU tests (not collected by pytest)."""
import functools
import sys

import numpy as np
import pytest

import oracle as O
import paper_1805_00280_amd as P
from paper_1805_00280_amd import workloads as WL


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@functools.lru_cache(maxsize=8)
def oracle_rmat(scale, ef, a, b, c, g, weighted):
    return O.rmat_csr(scale, ef, a, b, c, g, weighted=weighted, nthreads=16)


def gpu_graph_from_oracle(og, **kw):
    return P.Graph.from_numpy(og.off, og.adj, og.wt, **kw)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def starts_tensor(torch, starts):
    return torch.from_numpy(np.ascontiguousarray(starts, dtype=np.uint32).view(np.int32)).cuda()


def gpu_walk(g, starts_np, L, p, q, seed, walk_base=0, **opts):
    torch = torch_cuda()
    st = starts_tensor(torch, starts_np)
    out = g.walk(st, L, p, q, seed, walk_base=walk_base, **opts)
    torch.cuda.synchronize()
    return u32(out)


def oracle_walk(og, starts_np, L, p, q, seed, walk_base=0, d_rule=1024, a_cap=1024, wids=None, approx_t=0):
    return O.walk(og, starts_np, L, p, q, seed, walk_base=walk_base, wids=wids, d_rule=d_rule, a_cap=a_cap,
                  nthreads=16, approx_t=approx_t)["out"]


def first_mismatch(a, b):
    bad = np.nonzero(np.any(a != b, axis=1))[0]
    if len(bad) == 0:
        return None
    i = int(bad[0])
    return f"{len(bad)} rows differ; first row {i}:\n gpu    {a[i][:24].tolist()}\n oracle {b[i][:24].tolist()}"
