"""The C-ABI library loads and exports every symbol include/n2v.h declares
(CPU only: host-side queries, no device work)."""
import ctypes as C
import os
import re

import pytest

import paper_1805_00280_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    hdr = open(os.path.join(ROOT, "include", "n2v.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(n2v_\w+)\s*\(", hdr)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libn2v.so not built (run __graft_entry__.build())")
    return P.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTS) == names


def test_abi_version(lib):
    assert lib.n2v_abi_version() == 7


def test_defaults(lib):
    g = P.GraphOpts()
    lib.n2v_graph_opts_default(C.byref(g))
    assert (g.d_rule, g.a_cap, g.validate) == (1024, 1024, 1)
    o = P.exec_opts()
    assert o.mode == P.MODE_AUTO and o.t_wave <= 1024
    assert o.memo == 1 and o.t_wg == 65536 and o.search_ratio == 24
    s = P.ServerOpts()
    lib.n2v_server_opts_default(C.byref(s))
    assert s.chunk_walks > 0 and s.max_queue > 0


def test_rmat_workspace_query(lib):
    ws, mm = C.c_size_t(), C.c_uint64()
    prm = P.RmatParams(12, 16, 0.57, 0.19, 0.19, 12, 0)
    assert lib.n2v_rmat_workspace(C.byref(prm), C.byref(ws), C.byref(mm)) == 0
    assert mm.value == 2 * 16 * 4096
    assert ws.value >= 2 * 8 * mm.value
    bad = P.RmatParams(0, 16, 0.57, 0.19, 0.19, 12, 0)
    assert lib.n2v_rmat_workspace(C.byref(bad), C.byref(ws), C.byref(mm)) == -1
    assert b"bad parameters" in lib.n2v_last_error()
    bad = P.RmatParams(12, 16, 0.7, 0.2, 0.2, 12, 0)
    assert lib.n2v_rmat_workspace(C.byref(bad), C.byref(ws), C.byref(mm)) == -1


def test_graph_workspace_query(lib):
    ws = C.c_size_t()
    assert lib.n2v_graph_workspace(1000, 5000, 0, C.byref(ws)) == 0
    unweighted = ws.value
    assert unweighted >= 16 * 1000 + 8 * 5000
    assert lib.n2v_graph_workspace(1000, 5000, 1, C.byref(ws)) == 0
    assert ws.value > unweighted
    assert lib.n2v_graph_workspace(0, 5000, 0, C.byref(ws)) == -1


def test_null_arguments_rejected_without_device_work(lib):
    assert lib.n2v_walk_ex(None, None, 0, 0, 1, 1.0, 1.0, 0, None, 1, None, None, None, None, 0, None) == -1
    assert lib.n2v_graph_destroy(None) == 0
    assert lib.n2v_server_destroy(None) == 0
    assert lib.n2v_poll(None, 1, None) == -1


def test_memo_calls_reject_null_arguments(lib):
    dmin, b = C.c_uint32(), C.c_size_t()
    assert lib.n2v_graph_memo_plan(None, 0, C.byref(dmin), C.byref(b)) == -1
    assert lib.n2v_graph_set_memo_min(None, None, 0, 0) == -1
    assert lib.n2v_graph_memo_bytes(None, C.byref(b)) == -1
    assert lib.n2v_graph_memo_clear(None, None) == -1


def test_visit_profile_and_approx_reject_null_arguments(lib):
    assert lib.n2v_visit_profile(None, None, 1, 2, None, None, None) == -1
    assert lib.n2v_walk_approx(None, None, 0, 0, 10, C.c_float(1.0), C.c_float(1.0), 0, 1000, None, 1, None, None,
                               None, None, 0, None) == -1


def test_struct_layouts_match_the_header(tmp_path):
    # the binding's ctypes structs against the C compiler's view of include/n2v.h
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pairs = [("n2v_rmat_params", P.RmatParams), ("n2v_graph_opts", P.GraphOpts), ("n2v_exec_opts", P.ExecOpts),
             ("n2v_server_opts", P.ServerOpts), ("n2v_request", P.Request), ("n2v_result", P.Result),
             ("n2v_sgns_params", P.SgnsParams)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "n2v.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, cls in pairs:
        assert int(got[f"{cname} size"]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname} {f}"]) == getattr(cls, f).offset, (cname, f)
