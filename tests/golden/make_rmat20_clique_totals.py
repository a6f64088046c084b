"""Writes rmat20_clique_totals.json: the full K4 and K5 counts of the R-MAT
scale-20 graph (edge factor 16, (a,b,c,d) = (0.57,0.19,0.19,0.05), seed 2001),
computed by the oracle alone, for the GPU parity tests to compare the GPU's
full totals against.

The count of a pattern decomposes exactly over the roots of the first loop
(Theorem 1: every instance is found once, from one root), so the roots are
split round-robin over worker processes, each runs the oracle's plain
nested loops (its own schedule rule and every relation of Algorithm 1) over
its share, and the partial totals are summed in Python integers.

Run from the repository root:
    python tests/golden/make_rmat20_clique_totals.py [workers]
(about half an hour on 8 cores; rewrite only when the oracle's arithmetic or
the input generators change)."""

from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import patterns as P  # noqa: E402
from paper_1911_12877_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat20_clique_totals.json")
PATTERNS = ["k4", "k5"]

_G = None  # the prepared graph, inherited by forked workers


def _shard(args):
    name, w, n_workers = args
    roots = np.arange(w, _G.n, n_workers, dtype=np.int32)
    t0 = time.time()
    c = oracle.count(_G, P.named(name), True, roots=roots)
    return name, w, str(c), time.time() - t0


def main():
    global _G
    n_workers = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    t0 = time.time()
    _G = oracle.from_edge_tuple(synth.config_graph("rmat20"))
    print(f"rmat20 prepared in {time.time() - t0:.0f} s (n={_G.n}, nnz={_G.col.size})",
          flush=True)
    jobs = [(nm, w, n_workers) for nm in PATTERNS for w in range(n_workers)]
    totals = {nm: 0 for nm in PATTERNS}
    secs = {nm: 0.0 for nm in PATTERNS}
    with mp.get_context("fork").Pool(n_workers) as pool:
        for nm, w, c, dt in pool.imap_unordered(_shard, jobs):
            totals[nm] += int(c)
            secs[nm] += dt
            print(f"  {nm} shard {w}/{n_workers}: {c} in {dt:.0f} s", flush=True)
    out = {"graph": "rmat20", "induced": True, "workers": n_workers,
           "core_seconds": {nm: round(s, 1) for nm, s in secs.items()},
           "counts": {nm: str(v) for nm, v in totals.items()}}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT, out["counts"], flush=True)


if __name__ == "__main__":
    main()
