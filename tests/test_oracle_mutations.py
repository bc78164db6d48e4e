"""Planted mistakes in copies of the oracle are caught by the pins (CPU only).

Each case edits one line of a private copy of the oracle (oracle.c unless
another file is named), builds it under /tmp,
and runs a subset of the pin tests against it in a subprocess; the subset
must fail.  The committed oracle is never modified.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = [
    ("swap common and outward multipliers",
     "if (or_has_edge(g, t, x)) return w * A[1];", "if (or_has_edge(g, t, x)) return w * A[2];"),
    ("drop the return bias",
     "if (x == t) return w * A[0];", "if (x == t) return w * A[1];"),
    ("first move uses second-order weights",
     "if (s == 0) return w;", "if (s == 99) return w;"),
    ("inverse CDF off by one",
     "if (P > target) return g->adj[g->off[v] + j];", "if (P >= target) return g->adj[g->off[v] + j];"),
    ("envelope too small",
     "if (A[2] > amax) amax = A[2];\n        uint64_t E = (uint64_t)g->wmax[v] * (s == 0 ? 1u : amax);",
     "if (A[2] > amax) amax = A[2];\n        uint64_t E = (uint64_t)g->wmax[v] * (s == 0 ? 1u : A[1]);"),
    ("wrong Philox multiplier",
     "uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;", "uint64_t p1 = (uint64_t)0xCD9E8D57u * c1;"),
    ("R-MAT row and column bits transposed",
     "u |= (quad >> 1) << (scale - 1 - l);", "u |= (quad & 1u) << (scale - 1 - l);"),
    ("weight of the wrong pair",
     "ph(gseed, lo, hi, 0, 2, r);", "ph(gseed, lo, lo, 0, 2, r);"),
    ("FN-Approx: d_u common neighbours as Eq. 3 prints",
     "uint64_t cmax = du - 1 < dv - 1 ? du - 1 : dv - 1;", "uint64_t cmax = du < dv - 1 ? du : dv - 1;"),
    ("FN-Approx: return multiplier dropped",
     "uint64_t with_none = A[0] + (dv - 1) * A[2];", "uint64_t with_none = (dv - 1) * A[2];"),
    ("FN-Approx: numerator multipliers swapped",
     "*lb_num = wlo * a_lo;", "*lb_num = wlo * a_hi;"),
    ("FN-Approx: weight range ignored",
     "*ub_num = whi * a_hi;", "*ub_num = wlo * a_hi;"),
    ("FN-Approx: threshold compared the wrong way",
     "return (or_u128)T * diff < (or_u128)ud * ld;", "return (or_u128)T * diff > (or_u128)ud * ld;"),
    ("FN-Approx: popular previous vertex accepted",
     "if (dv <= d_rule || du > d_rule || du == 0) return 0;", "if (dv <= d_rule || du == 0) return 0;"),
    ("FN-Approx: draw from the second-order law",
     "if (s > 0 && or_approx_applies(g, t, v, A, d_rule, approx_t)) return or_static_draw(g, seed, wid, s, v);",
     "if (s > 0 && or_approx_applies(g, t, v, A, d_rule, approx_t)) return or_inverse_cdf(g, seed, wid, s, 0, t, v, A);"),
    # the isolated algorithmic-bytes model
    ("cost: off[v+1] not charged",
     "    seg_add(&S, SEG_OFF, (uint64_t)v * 8 + 8);", "    (void)0;"),
    ("cost: merge branch drops N(t)",
     "    if (s > 0) seg_add_range(&D, SEG_ADJ, ot * 4, (ot + dt) * 4);",
     "    if (s > 99) seg_add_range(&D, SEG_ADJ, ot * 4, (ot + dt) * 4);"),
    ("cost: search probes not charged",
     "        seg_add(s, SEG_ADJ, mid * 4);", "        (void)mid;"),
    ("cost: sparse branch searches the wrong row",
     "            uint64_t pos = seg_search(&P, g->adj, ov, ov + d, y);",
     "            uint64_t pos = seg_search(&P, g->adj, ot, ot + dt, y);"),
    ("cost: FN-Approx move charged as exact",
     "    if (s > 0 && or_approx_applies(g, t, v, A, d_rule, approx_t)) {\n        /* first-order draw",
     "    if (s > 99 && or_approx_applies(g, t, v, A, d_rule, approx_t)) {\n        /* first-order draw"),
    ("cost: weight of a proposal not charged",
     "if (g->wt) { seg_add(&S, SEG_WT, (ov + j) * 2); w = g->wt[ov + j]; }", "if (g->wt) { w = g->wt[ov + j]; }"),
    # the checksum hash
    ("checksum: column and vertex counter words swapped",
     "ph(seed, wid, col, x, 3, r);", "ph(seed, wid, x, col, 3, r);"),
    # the memo-aware model
    ("memo: summary row not charged",
     "    return row + (4 * h + 63) / 64 + (4 * ht + 63) / 64;", "    return (4 * h + 63) / 64 + (4 * ht + 63) / 64;"),
    ("memo: summary row segments not rounded up to even",
     "    segs = (segs + 1) & ~1ull;", "    segs = segs;"),
    ("memo: summary row of 64 segments at every degree",
     "    uint64_t segs = (tiles + per - 1) / per;", "    uint64_t segs = 64;"),
    ("memo: tiles per summary segment off by one",
     "    uint64_t per = tiles ? (tiles + 63) / 64 : 1;", "    uint64_t per = tiles ? (tiles + 63) / 64 + 1 : 1;"),
    ("memo: one summary per direction of a pair",
     "key = t < v ? ((uint64_t)t << 32) | v : ((uint64_t)v << 32) | t;", "key = ((uint64_t)v << 32) | t;"),
    ("memo: intersection charged on every move",
     "if (k > 0 && keys[k] == keys[k - 1]) continue;", "if (0) continue;"),
    ("memo: line of off[v+1] dropped",
     "return lines_of(8, v, (uint64_t)v + 2);", "return lines_of(8, v, (uint64_t)v + 1);"),
    ("memo: search levels off by one",
     "while ((16ull << k) < d) ++k;", "while ((16ull << k) <= d) ++k;"),
    ("memo: weighted summaries shared by both directions",
     "if (!weighted && or_memo_keeps(dt, memo_min))", "if (or_memo_keeps(dt, memo_min))"),
    ("memo: weighted summary row charged as unweighted",
     "    return (weighted ? 22 : 6) * segs;", "    return 6 * segs;"),
    ("memo: summary read even when dearer",
     "            if (warm < cold) {", "            if (warm < cold + 1000000) {"),
    # the Skip-gram step that consumes the walks
    ("sgns: negatives drawn with another counter tag",
     "ph(seed, (uint32_t)(walk_base + i), k, step, 6, r);", "ph(seed, (uint32_t)(walk_base + i), k, step, 5, r);"),
    ("sgns: a center is its own context",
     "pos = (dist >= 1) & (dist <= window)", "pos = dist <= window", "skipgram.py"),
    ("sgns: context window one short",
     "pos = (dist >= 1) & (dist <= window)", "pos = (dist >= 1) & (dist < window)", "skipgram.py"),
    ("sgns: negative weight missing from the gradient",
     "G[:, n:] = neg_weight * sigmoid(Z[:, n:])", "G[:, n:] = sigmoid(Z[:, n:])", "skipgram.py"),
    ("sgns: context gradient with the wrong sign",
     "np.where(pos, sigmoid(Z[:, :n]) - 1.0, 0.0)", "np.where(pos, 1.0 - sigmoid(Z[:, :n]), 0.0)", "skipgram.py"),
    ("sgns: target gradient from the wrong vectors",
     "np.add.at(gout, tids, G.T @ V)", "np.add.at(gout, tids, G.T @ (0.5 * V))", "skipgram.py"),
    ("sgns: occurrences not counted per target",
     "np.add.at(cout, tids, 1.0)", "cout[tids] += 1.0", "skipgram.py"),
]

TESTS = ["tests/test_oracle_philox.py", "tests/test_oracle_rmat.py", "tests/test_oracle_law.py",
         "tests/test_oracle_invariants.py", "tests/test_oracle_approx.py", "tests/test_oracle_cost.py",
         "tests/test_oracle_skipgram.py"]


@pytest.mark.parametrize("mutation", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(mutation):
    name, old, new = mutation[:3]
    fname = mutation[3] if len(mutation) > 3 else "oracle.c"
    path = os.path.join(ROOT, "oracle", fname)
    src = open(path).read()
    assert src.count(old) == 1, name
    tmp = tempfile.mkdtemp(prefix="n2v_mut_")
    try:
        pkg = os.path.join(tmp, "oracle")
        shutil.copytree(os.path.join(ROOT, "oracle"), pkg,
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
        with open(os.path.join(pkg, fname), "w") as f:
            f.write(src.replace(old, new))
        subprocess.check_call([sys.executable, os.path.join(pkg, "build.py")],
                              stdout=subprocess.DEVNULL)
        tdir = os.path.join(tmp, "tests")
        shutil.copytree(os.path.join(ROOT, "tests"), tdir,
                        ignore=shutil.ignore_patterns("__pycache__", "test_oracle_mutations.py"))
        env = dict(os.environ, PYTHONPATH=tmp)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "-m", "not gpu"] + [os.path.join(tmp, t) for t in TESTS],
                           cwd=tmp, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                           timeout=600)
        assert r.returncode != 0, f"mutation '{name}' was not caught:\n" + r.stdout.decode()[-2000:]
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
