"""bench.py's torch evaluation of the memo-aware bytes model equals the oracle's
or_memo_pass_bytes on the oracle's own walks (CPU tensors; no GPU needed)."""
import os
import sys

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("weighted,d_rule,memo_min", [(False, 40, 41), (False, 40, 120), (False, 40, None),
                                                      (True, 40, 41), (False, 1024, 1025)])
def test_torch_pass_bytes_equal_the_oracle(weighted, d_rule, memo_min):
    import torch
    g = O.rmat_csr(13, 16, 0.65, 0.15, 0.15, 13, weighted=weighted)
    starts = np.tile(np.arange(g.n, dtype=np.uint32), 2)
    out = O.walk(g, starts, 15, 0.25, 4.0, 5, d_rule=d_rule)["out"]
    want = O.memo_pass_bytes(g.off, out, 15, d_rule=d_rule, memo_min=memo_min if memo_min else d_rule + 1,
                             memo=memo_min is not None, weighted=weighted)
    cold = O.memo_pass_bytes(g.off, out, 15, d_rule=d_rule, memo=False, weighted=weighted)
    got = bench.pass_bytes(torch.from_numpy(g.off.view(np.int64)), torch.from_numpy(out.view(np.int32)), 15,
                           d_rule, memo_min, weighted)
    assert got["hub_bytes"] == want["hub_bytes"]
    assert got["hub_bytes_cold"] == cold["hub_bytes"]
    assert got["hub_moves"] == want["hub_moves"] and got["other_moves"] == want["other_moves"]
    assert got["warm_moves"] == want["warm_moves"] and got["intersections"] == want["intersections"]
    if memo_min == 41:
        assert want["warm_moves"] > 0 or weighted
