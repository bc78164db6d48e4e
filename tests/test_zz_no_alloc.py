"""n2v_walk_static (plain form in the library's static scratch, no allocation)
against n2v_walk_ex on the same inputs: two calls in a row, the second smaller."""
import ctypes as C

import numpy as np
import pytest

import paper_1805_00280_amd as P
from gpuhelp import (first_mismatch, gpu_graph_from_oracle, oracle_rmat, oracle_walk, say, starts_tensor,
                     torch_cuda, u32)

pytestmark = pytest.mark.gpu


def static_walk(g, st, L, p, q, seed, walk_base=0, approx_t=0):
    torch = torch_cuda()
    n = int(st.numel())
    out = torch.full((n, L + 1), -7, dtype=torch.int32, device="cuda")
    o = P.exec_opts(g)
    rc = P.lib().n2v_walk_static(g._h, C.c_void_p(st.data_ptr()), n, walk_base, L, p, q, seed, approx_t,
                                 C.byref(o), P.OUT_WALKS, C.c_void_p(out.data_ptr()), None, None,
                                 P._stream(None))
    assert rc == 0, P.lib().n2v_last_error()
    torch.cuda.synchronize()
    return u32(out)


def ex_walk(g, st, L, p, q, seed, mode, walk_base=0, approx_t=0):
    torch = torch_cuda()
    out = g.walk(st, L, p, q, seed, walk_base=walk_base, mode=mode, approx_t=approx_t)
    torch.cuda.synchronize()
    return u32(out)


@pytest.mark.parametrize("memo", [False, True])
def test_static_scratch_equals_the_workspace_entry_point(memo):
    torch = torch_cuda()
    og = oracle_rmat(13, 16, 0.65, 0.15, 0.15, 29, False)
    g = gpu_graph_from_oracle(og, d_rule=40)
    if memo:
        g.attach_memo()
    rng = np.random.default_rng(3)
    # a large call, then a smaller one with other parameters: the second must not see the
    # first's state or counters
    calls = [(np.tile(np.arange(og.n, dtype=np.uint32), 3), 40, 0.25, 4.0, 11, 0, 0),
             (rng.integers(0, og.n, size=1500).astype(np.uint32), 25, 2.0, 0.5, 12, 1 << 20, 50)]
    for starts, L, p, q, seed, base, approx_t in calls:
        st = starts_tensor(torch, starts)
        say(f"[no-alloc] memo={memo} walks={len(starts)} L={L} p={p} q={q} approx={approx_t}")
        got = static_walk(g, st, L, p, q, seed, base, approx_t)
        for mode in (P.MODE_PLAIN, P.MODE_PERSISTENT):
            want = ex_walk(g, st, L, p, q, seed, mode, base, approx_t)
            assert first_mismatch(got, want) is None, (mode, first_mismatch(got, want))
        ref = oracle_walk(og, starts, L, p, q, seed, walk_base=base, d_rule=40, approx_t=approx_t)
        assert first_mismatch(got, ref) is None
    if memo:
        g.detach_memo()


def test_static_scratch_limits_are_refused_before_any_launch():
    torch = torch_cuda()
    og = oracle_rmat(10, 16, 0.57, 0.19, 0.19, 10, False)
    g = gpu_graph_from_oracle(og)
    o = P.exec_opts(g)
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    out = torch.zeros(4 * 1025, dtype=torch.int32, device="cuda")
    rc = P.lib().n2v_walk_static(g._h, C.c_void_p(st.data_ptr()), (1 << 21) + 1, 0, 10, 1.0, 1.0, 1, 0, C.byref(o),
                                 P.OUT_WALKS, C.c_void_p(out.data_ptr()), None, None, P._stream(None))
    assert rc == -2 and b"static scratch" in P.lib().n2v_last_error()
    rc = P.lib().n2v_walk_static(g._h, C.c_void_p(st.data_ptr()), 4, 0, 1024, 1.0, 1.0, 1, 0, C.byref(o),
                                 P.OUT_WALKS, C.c_void_p(out.data_ptr()), None, None, P._stream(None))
    assert rc == -2
    torch.cuda.synchronize()
    assert int(out.abs().sum().item()) == 0
