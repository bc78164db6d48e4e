"""Skip-gram with negative sampling over walks: plain fp64 reference (test
infrastructure only; imported by the test suite and the benchmark's CPU leg).

node2vec learns vertex embeddings by running Skip-gram over its walks
(Sections 1 and 2.1 of the paper).  One training step, written out from its
definition (word2vec's Skip-gram with negative sampling, with each walk's
negatives shared by all of its centers):
  - each position i before the walk's first sentinel is a center with vector
    v = win[x_i]; its contexts are the positions j with 1 <= |i - j| <= window
    (u = wout[x_j]); the walk's negatives n_k (u = wout[n_k]) are negatives of
    every center;
  - z = v . u; loss = sum over (center, context) of log(1 + exp(-z)) plus
    neg_weight times the sum over (center, negative) of log(1 + exp(z));
  - the gradient of that loss: d/dz = sigmoid(z) - 1 for a context and
    neg_weight * sigmoid(z) for a negative, times u for the center's vector
    and times v for the target's, summed over the whole batch;
  - after the whole batch, each row moves by lr times its mean gradient per
    occurrence in the batch: w[x] -= lr * dL/dw[x] / (occurrences of x as a
    center, resp. as a target, at least 1).
Negatives come from the oracle's C draw (or_sgns_negatives: Philox and the
cumulative noise table).  Shares nothing with the GPU library.
"""
from __future__ import annotations

import numpy as np

from . import SENT, _load, _ptr


def negatives(cum, seed, walk_base, n_walks, nneg, step):
    """The walks' negatives (n_walks x nneg, uint32)."""
    import ctypes as C
    lib = _load()
    if not hasattr(lib, "_sgns_set"):
        lib.or_sgns_negatives.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                          C.c_uint32, C.c_void_p]
        lib.or_sgns_negatives.restype = None
        lib._sgns_set = True
    cum = np.ascontiguousarray(cum, dtype=np.uint64)
    out = np.zeros((n_walks, nneg), dtype=np.uint32)
    lib.or_sgns_negatives(_ptr(cum), len(cum) - 1, seed, walk_base, step, n_walks, nneg, _ptr(out))
    return out


def walk_length(row):
    """Entries before the first sentinel."""
    s = np.nonzero(np.asarray(row, dtype=np.uint32) == SENT)[0]
    return int(s[0]) if len(s) else len(row)


def softplus(x):
    return np.logaddexp(0.0, x)


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def step(win, wout, walks, negs, window, neg_weight, lr):
    """One step; returns (new win, new wout, loss, gradient of win, gradient of wout,
    occurrences as centers, occurrences as targets), fp64."""
    win = np.asarray(win, dtype=np.float64)
    wout = np.asarray(wout, dtype=np.float64)
    gin = np.zeros_like(win)
    gout = np.zeros_like(wout)
    cin = np.zeros(len(win))
    cout = np.zeros(len(wout))
    loss = 0.0
    for w, row in enumerate(np.asarray(walks, dtype=np.uint32)):
        n = walk_length(row)
        if n == 0:
            continue
        ids = row[:n].astype(np.int64)
        neg = np.asarray(negs[w], dtype=np.int64)
        tids = np.concatenate([ids, neg])
        V = win[ids]
        T = wout[tids]
        Z = V @ T.T
        i = np.arange(n)[:, None]
        j = np.arange(n)[None, :]
        dist = np.abs(i - j)
        pos = (dist >= 1) & (dist <= window)
        G = np.zeros_like(Z)
        G[:, :n] = np.where(pos, sigmoid(Z[:, :n]) - 1.0, 0.0)
        G[:, n:] = neg_weight * sigmoid(Z[:, n:])
        loss += float(softplus(-Z[:, :n])[pos].sum() + neg_weight * softplus(Z[:, n:]).sum())
        np.add.at(gin, ids, G @ T)
        np.add.at(gout, tids, G.T @ V)
        np.add.at(cin, ids, 1.0)
        np.add.at(cout, tids, 1.0)
    sin = lr / np.maximum(cin, 1.0)
    sout = lr / np.maximum(cout, 1.0)
    return win - sin[:, None] * gin, wout - sout[:, None] * gout, loss, gin, gout, cin, cout
