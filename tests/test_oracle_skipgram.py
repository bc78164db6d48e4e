"""Pins of the oracle's Skip-gram step (CPU): the gradient against finite
differences of the loss, the loss at zero embeddings by counting pairs by hand,
a two-vertex walk by hand, and the negative draw against the Python Philox."""
import math

import numpy as np

import oracle as O
from oracle import skipgram as SG
from oracle.philox_ref import philox4x32

S = O.SENT


def test_gradient_is_the_derivative_of_the_loss():
    rng = np.random.default_rng(1)
    n, D = 6, 3
    win, wout = rng.normal(size=(n, D)), rng.normal(size=(n, D))
    walks = np.array([[0, 1, 2, 3, S], [4, 2, 2, 5, 1]], dtype=np.uint32)
    negs = np.array([[5, 3], [0, 0]], dtype=np.uint32)

    def loss(a, b):
        return SG.step(a, b, walks, negs, 2, 0.7, 0.0)[2]

    _, _, L0, gin, gout, cin, cout = SG.step(win, wout, walks, negs, 2, 0.7, 0.0)
    h = 1e-6
    for table, grad, which in ((win, gin, 0), (wout, gout, 1)):
        num = np.zeros_like(table)
        for idx in np.ndindex(table.shape):
            a, b = table.copy(), table.copy()
            a[idx] += h
            b[idx] -= h
            lp = loss(a, wout) if which == 0 else loss(win, a)
            lm = loss(b, wout) if which == 0 else loss(win, b)
            num[idx] = (lp - lm) / (2 * h)
        assert np.allclose(grad, num, rtol=1e-6, atol=1e-7), which
    # the step moves each row against its mean gradient per occurrence
    nwin, nwout = SG.step(win, wout, walks, negs, 2, 0.7, 0.1)[:2]
    assert np.allclose(nwin, win - 0.1 * gin / np.maximum(cin, 1)[:, None])
    assert np.allclose(nwout, wout - 0.1 * gout / np.maximum(cout, 1)[:, None])
    assert loss(nwin, nwout) < L0


def test_occurrences_by_hand():
    # walk [0, 1, 0, 2], window 1, negatives (3, 3): vertex 0 is a center twice, 1 and 2 once;
    # as targets 0 appears twice, 1 and 2 once, 3 twice (one per negative slot)
    rng = np.random.default_rng(7)
    win, wout = rng.normal(size=(4, 3)), rng.normal(size=(4, 3))
    walks = np.array([[0, 1, 0, 2]], dtype=np.uint32)
    negs = np.array([[3, 3]], dtype=np.uint32)
    nwin, nwout, _, gin, gout, cin, cout = SG.step(win, wout, walks, negs, 1, 0.5, 0.2)
    assert cin.tolist() == [2, 1, 1, 0] and cout.tolist() == [2, 1, 1, 2]
    assert np.allclose(nwin[0], win[0] - 0.2 * gin[0] / 2) and np.allclose(nwin[3], win[3])
    assert np.allclose(nwout[3], wout[3] - 0.2 * gout[3] / 2)


def test_loss_at_zero_embeddings_counts_the_pairs():
    # z = 0 everywhere: every term is log 2.  Walk of 5, window 2: contexts per position
    # 2, 3, 4, 3, 2 = 14 pairs; 5 centers x 3 negatives = 15 pairs
    z = np.zeros((8, 4))
    walks = np.array([[1, 2, 3, 4, 5, S, S]], dtype=np.uint32)
    negs = np.array([[6, 7, 0]], dtype=np.uint32)
    _, _, L, gin, gout = SG.step(z, z, walks, negs, 2, 0.25, 1.0)[:5]
    assert math.isclose(L, math.log(2) * (14 + 0.25 * 15), rel_tol=1e-12)
    assert not gin.any() and not gout.any()  # zero vectors give zero gradients


def test_two_vertex_walk_by_hand():
    # walk [0, 1], window 1, no negatives: loss = softplus(-v0.u1) + softplus(-v1.u0),
    # dL/dv0 = (sigmoid(v0.u1) - 1) u1, dL/du1 = (sigmoid(v0.u1) - 1) v0, and likewise
    win = np.array([[1.0, 2.0], [0.5, -1.0]])
    wout = np.array([[-0.5, 0.25], [2.0, 1.0]])
    walks = np.array([[0, 1]], dtype=np.uint32)
    negs = np.zeros((1, 0), dtype=np.uint32)
    _, _, L, gin, gout = SG.step(win, wout, walks, negs, 1, 1.0, 0.0)[:5]
    z01 = 1.0 * 2.0 + 2.0 * 1.0      # v0 . u1 = 4
    z10 = 0.5 * -0.5 + -1.0 * 0.25   # v1 . u0 = -0.5
    sp = lambda x: math.log1p(math.exp(x))
    sg = lambda x: 1.0 / (1.0 + math.exp(-x))
    assert math.isclose(L, sp(-z01) + sp(-z10), rel_tol=1e-12)
    assert np.allclose(gin[0], (sg(z01) - 1) * wout[1]) and np.allclose(gin[1], (sg(z10) - 1) * wout[0])
    assert np.allclose(gout[1], (sg(z01) - 1) * win[0]) and np.allclose(gout[0], (sg(z10) - 1) * win[1])


def test_negative_draw_against_the_python_philox():
    w = np.array([3, 0, 5, 1, 0, 7], dtype=np.uint64)
    cum = np.concatenate([[0], np.cumsum(w)]).astype(np.uint64)
    seed, base, step = 0xABCDEF0123, 1000, 7
    got = SG.negatives(cum, seed, base, 50, 9, step)
    for i in range(50):
        for k in range(9):
            r = philox4x32((seed & 0xFFFFFFFF, seed >> 32), (base + i, k, step, 6))
            target = (((r[0] << 32) | r[1]) * int(cum[-1])) >> 64
            x = int(np.searchsorted(cum, target, side="right")) - 1
            assert got[i, k] == x
    big = SG.negatives(cum, seed, 0, 20000, 4, 0).ravel()
    freq = np.bincount(big, minlength=6) / len(big)
    assert freq[1] == 0 and freq[4] == 0
    assert np.allclose(freq, w / w.sum(), atol=0.01)


def test_sentinel_tail_is_ignored():
    rng = np.random.default_rng(4)
    win, wout = rng.normal(size=(5, 3)), rng.normal(size=(5, 3))
    negs = np.array([[4]], dtype=np.uint32)
    a = SG.step(win, wout, np.array([[0, 1, 2, S, S]], dtype=np.uint32), negs, 2, 0.5, 0.1)
    b = SG.step(win, wout, np.array([[0, 1, 2]], dtype=np.uint32), negs, 2, 0.5, 0.1)
    for x, y in zip(a, b):
        assert np.allclose(x, y)
