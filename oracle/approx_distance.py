"""Distance of FN-Approx from the exact law (test infrastructure only).

For one workload, runs a seeded sample of walks through the oracle with
FN-Approx (Section 3.4), collects every move the approximation replaced (a
move at a vertex v of degree > d_rule after a vertex t of degree <= d_rule
whose bound gap is below the threshold) and computes, for each, the total
variation distance between the exact second-order law at (t, v) (weights
w_vx times 1/p, 1 or 1/q by the distance of x from t) and the static-weight
law drawn instead.  Prints one JSON line.

    python -m oracle.approx_distance skew5 --pq 0.5,2 --approx 1000 --walks 2000
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle as O  # noqa: E402
from paper_1805_00280_amd import workloads as WL  # noqa: E402


def tv_distance(og, t, v, p, q):
    """Total variation between the exact law at (t, v) and w / sum(w)."""
    nv = og.adj[int(og.off[v]):int(og.off[v + 1])]
    nt = og.adj[int(og.off[t]):int(og.off[t + 1])]
    w = np.ones(len(nv)) if og.wt is None else og.wt[int(og.off[v]):int(og.off[v + 1])].astype(np.float64)
    alpha = np.where(np.isin(nv, nt), 1.0, 1.0 / q)
    alpha[nv == t] = 1.0 / p
    exact = w * alpha / np.sum(w * alpha)
    return 0.5 * float(np.abs(exact - w / w.sum()).sum())


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("workload", help="skew<S>, wec<K> or er<K>")
    ap.add_argument("--pq", default="0.5,2")
    ap.add_argument("--approx", type=int, default=1000)
    ap.add_argument("--walks", type=int, default=2000)
    ap.add_argument("--threads", type=int, default=8)
    args = ap.parse_args()
    p, q = (float(x) for x in args.pq.split(","))
    w = WL.paper_family(args.workload, p, q)
    og = O.rmat_csr(*w.rmat_args(), weighted=w.weighted, nthreads=args.threads)
    ids = w.sample_walk_ids(args.walks, seed=21)
    out = O.walk(og, (ids % w.n).astype(np.uint32), w.L, p, q, w.seed, wids=ids, approx_t=args.approx,
                 nthreads=args.threads)["out"]
    moves, tvs, degs = 0, [], []
    for row in out:
        for c in range(2, w.L + 1):
            t, v = int(row[c - 2]), int(row[c - 1])
            if row[c] == O.SENT:
                break
            moves += 1
            if O.approx_applies(og, t, v, p, q, args.approx):
                tvs.append(tv_distance(og, t, v, p, q))
                degs.append(int(og.off[v + 1] - og.off[v]))
    tvs = np.array(tvs) if tvs else np.zeros(0)
    res = {"workload": w.name, "approx_t": args.approx, "walks": len(ids), "second_order_moves": moves,
           "approximated_moves": int(len(tvs)), "approximated_share": len(tvs) / max(moves, 1),
           "tv_mean": float(tvs.mean()) if len(tvs) else None,
           "tv_p99": float(np.percentile(tvs, 99)) if len(tvs) else None,
           "tv_max": float(tvs.max()) if len(tvs) else None,
           "min_degree_approximated": min(degs) if degs else None}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
