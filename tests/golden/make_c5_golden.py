#!/usr/bin/env python3
"""Writes c5_hypergraphs_r128.json: the oracle's solution of every graph of
the random relation hypergraph workload (256 graphs, 8-14 variables,
relation arity 2-3, 2-4 exposed, 128 cells per axis, [-3,3]), as the number
of set entries and the SHA-256 of the output array (one byte per entry,
row-major over the exposed variables in their listed order).

Only the oracle computes: corner plots of every relation (orc_plot), then the
cluster tree of oracle.planner.bounded_merges executed by
oracle.solve_pairwise.  The instance generator is the shared input module;
each record carries the instance's SHA-256 so a changed generator is caught.

Usage: python tests/golden/make_c5_golden.py [n_graphs] (about 10 minutes on
8 cores for 256 graphs).
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import planner  # noqa: E402
from paper_1609_00061_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "c5_hypergraphs_r128.json")


def solve(s):
    res = {v: s.axes[v][2] for v in range(len(s.axes))}
    packs = [r.vars for r in s.relations]
    merges = planner.bounded_merges(packs, s.exposed, res)
    if merges is None:
        raise RuntimeError(f"{s.name}: no tree within the caps (the generator should have rejected it)")
    plots = [oracle.plot(r, s.axes)[0] for r in s.relations]
    return oracle.solve_pairwise(res, packs, plots, s.exposed, merges)


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    graphs = inputs.config5(n_graphs=n, index=0, res=128)
    recs = []
    t0 = time.time()
    for s in graphs:
        ref = np.ascontiguousarray(solve(s), dtype=np.uint8)
        recs.append({"name": s.name, "instance_sha256": s.digest(), "shape": list(ref.shape),
                     "nnz": int(ref.sum()), "sha256": hashlib.sha256(ref.tobytes()).hexdigest()})
        print(f"{s.name}: nnz {recs[-1]['nnz']} ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        json.dump({"workload": "config5(n_graphs=%d, index=0, res=128)" % n,
                   "output_hash": "sha256 of the uint8 array (one byte per entry, C order, exposed order)",
                   "graphs": recs}, f, indent=0)
        f.write("\n")


if __name__ == "__main__":
    main()
