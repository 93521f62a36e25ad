"""Counts the operations of the paper's closed form on the headline workload.

MEASUREMENT INFRASTRUCTURE, calling only oracle/ (the instrumented
closed-form oracle, opcount.cpp).  Writes op_count_covering_1M_p3_c2.json
next to this file, which bench.py reads for the algorithmic flops of its
roofline: the mean number of additions, multiplications, divisions, square
roots and transcendental calls per particle-triangle pair, overall and per
case of the dispatch of Sec. 4.6 (vertices inside the support), over every
pair of a seeded sample of the workload's particles.

Usage: python oracle/count_ops.py [--particles 2000]
"""
import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_2507_21686_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "op_count_covering_1M_p3_c2.json")


def pairs_of(wl, sel):
    """(particle index, triangle index) of every pair of the selected particles
    (dist < h, brute force against all triangles)."""
    out_i, out_t = [], []
    for i in sel:
        # candidates: a vertex within 4h in both coordinates (triangles are at most ~3h across)
        cand = np.nonzero((np.abs(wl.tri[0::2] - wl.px[i]).min(0) < 4 * wl.h) &
                          (np.abs(wl.tri[1::2] - wl.py[i]).min(0) < 4 * wl.h))[0]
        d2 = np.array([oracle.point_triangle_dist2(wl.px[i], wl.py[i], wl.tri[:, t]) for t in cand])
        for t in cand[d2 < wl.h * wl.h]:
            out_i.append(i)
            out_t.append(t)
    return np.array(out_i), np.array(out_t)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--particles", type=int, default=2000)
    args = ap.parse_args()
    wl = W.covering_workload()
    sel = np.sort(np.random.default_rng(0).choice(wl.n_particles, args.particles, replace=False))
    pi, pt = pairs_of(wl, sel)
    tri = wl.tri[:, pt].copy()
    tri[0::2] -= wl.px[pi]
    tri[1::2] -= wl.py[pi]
    tri /= wl.h
    counts, cls, _ = oracle.opcount_pairs(wl.kernel, tri, wl.nodal[:, pt])
    kinds = list(oracle.OPCOUNT_KINDS)

    def summary(c):
        d = {k: float(c[:, j].mean()) for j, k in enumerate(kinds)}
        d["fma"] = 0.0
        d["total"] = float(c.sum(1).mean())
        return d

    by_case = {}
    for k in range(4):
        m = cls == k
        if m.any():
            by_case[f"{k}_vertices_inside"] = dict(summary(counts[m]), fraction=float(m.mean()))
    res = {"workload": "covering mesh, 1,048,576 particles (jittered 1024^2 grid, seed 2), 65,536 triangles, "
                       "cubic Lagrange field, Wendland C2, h = 2.5/1024",
           "sample": f"every pair of {len(sel)} seeded random particles ({len(pi)} pairs)",
           "per_pair": summary(counts), "by_case": by_case,
           "counted": "add (incl. subtract), mul, div, sqrt, transcendental (log, atan2, cos, sin), each one "
                      "operation; the closed form has no fused multiply-add; operations between constants are "
                      "not counted; moment tables formed only to the degree the contraction reads",
           "written_by": "oracle/count_ops.py"}
    json.dump(res, open(OUT, "w"), indent=1)
    print(json.dumps(res["per_pair"]))


if __name__ == "__main__":
    main()
