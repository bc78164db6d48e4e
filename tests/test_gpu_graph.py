"""GPU R-MAT generator and graph creation against the oracle (bit-exact)."""
import numpy as np
import pytest

import paper_1805_00280_amd as P
from gpuhelp import oracle_rmat, say, torch_cuda, u32

pytestmark = pytest.mark.gpu

CASES = [
    (8, (0.57, 0.19, 0.19), False),
    (12, (0.57, 0.19, 0.19), False),   # the scale-12 walk workload's graph
    (14, (0.65, 0.15, 0.15), True),
    (16, (0.65, 0.15, 0.15), False),
    (20, (0.57, 0.19, 0.19), True),    # the scale-20 weighted walk workload's graph
]


@pytest.mark.parametrize("scale,abc,weighted", CASES)
def test_rmat_csr_bit_exact(scale, abc, weighted):
    torch = torch_cuda()
    say(f"[rmat] scale={scale} abc={abc} weighted={weighted}")
    off, adj, wt = P.Graph.generate_rmat(scale, 16, *abc, scale, weighted=weighted)
    torch.cuda.synchronize()
    og = oracle_rmat(scale, 16, *abc, scale, weighted)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), og.off)
    assert np.array_equal(u32(adj), og.adj)
    if weighted:
        assert np.array_equal(wt.cpu().numpy().view(np.uint16), og.wt)
    else:
        assert wt is None


def test_rmat_seed_changes_graph():
    torch = torch_cuda()
    _, a1, _ = P.Graph.generate_rmat(10, 8, 0.57, 0.19, 0.19, 1)
    _, a2, _ = P.Graph.generate_rmat(10, 8, 0.57, 0.19, 0.19, 2)
    torch.cuda.synchronize()
    assert a1.numel() != a2.numel() or not torch.equal(a1, a2)


def _csr(rows, n):
    off = np.zeros(n + 1, dtype=np.uint64)
    adj = []
    for v in range(n):
        adj.extend(rows.get(v, []))
        off[v + 1] = len(adj)
    return off, np.array(adj, dtype=np.uint32)


@pytest.mark.parametrize("name,rows,n,wt", [
    ("unsorted row", {0: [2, 1], 1: [0], 2: [0]}, 3, None),
    ("duplicate entry", {0: [1, 1], 1: [0]}, 2, None),
    ("self loop", {0: [0, 1], 1: [0]}, 2, None),
    ("id out of range", {0: [5], 1: [0]}, 2, None),
    ("zero weight", {0: [1], 1: [0]}, 2, [0, 1]),
])
def test_graph_create_rejects_bad_csr(name, rows, n, wt):
    torch_cuda()
    off, adj = _csr(rows, n)
    w = None if wt is None else np.array(wt, dtype=np.uint16)
    with pytest.raises(P.N2VError) as e:
        P.Graph.from_numpy(off, adj, w)
    assert e.value.code == -3, name


def test_graph_create_rejects_bad_offsets():
    torch_cuda()
    off = np.array([0, 2, 1, 3], dtype=np.uint64)
    adj = np.array([1, 2, 0], dtype=np.uint32)
    with pytest.raises(P.N2VError) as e:
        P.Graph.from_numpy(off, adj)
    assert e.value.code == -3


def test_symmetry_check_optional():
    torch_cuda()
    off, adj = _csr({0: [1], 1: [2], 2: []}, 3)  # directed path
    P.Graph.from_numpy(off, adj)  # accepted: directed graphs are allowed
    with pytest.raises(P.N2VError) as e:
        P.Graph.from_numpy(off, adj, validate=2)
    assert e.value.code == -3


def test_graph_info():
    torch_cuda()
    off, adj = _csr({0: [1], 1: [0]}, 2)
    g = P.Graph.from_numpy(off, adj, d_rule=7, a_cap=3)
    assert g.info() == {"n": 2, "m": 2, "d_rule": 7, "a_cap": 3, "weighted": False}
