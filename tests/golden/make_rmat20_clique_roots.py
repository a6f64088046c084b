"""Writes rmat20_clique_roots.json: per-root K4 and K5 counts of the R-MAT
scale-20 graph (edge factor 16, (a,b,c,d) = (0.57,0.19,0.19,0.05), seed 2001)
at roots chosen by their first-loop candidate count lo (the neighbours with a
smaller id after the degree reindex), computed by the oracle alone, for the
GPU parity tests.

The clique kernels put a root's candidates in bit rows of ceil(lo / 64)
words, in size classes of at most 2, 4 and 8 words and the rest.  Roots:
  * the 16 roots of largest lo (the widest class, rows of 9-11 words);
  * 8 seeded roots from each lo range (64,128], (128,256], (256,512] and
    (512, max];
  * the top-degree roots: ids 0..999 for K4, ids 0..99 for K5 (a K5 root of
    the widest class costs the oracle about two minutes).
Schedule: the analytic pick (the identity order for cliques) with Theorem 2's
single bound per loop, as the GPU runs it; a per-root count is the number of
cliques whose largest id is that root.

Run from the repository root:  python tests/golden/make_rmat20_clique_roots.py [workers]
(about 10 minutes on 8 cores)."""

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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat20_clique_roots.json")
CLASSES = [(64, 128), (128, 256), (256, 512), (512, 1 << 30)]

_G = None


def _one(args):
    name, root = args
    adj = P.named(name)
    order = P.pick_schedule(adj, True)[0]
    _, per = oracle.count(_G, adj, True, order=order, relations="thm2",
                          roots=np.array([root], np.int32), per_root=True)
    return name, int(root), str(int(per[0]))


def main():
    global _G
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    t0 = time.time()
    _G = oracle.from_edge_tuple(synth.config_graph("rmat20"))
    lo = oracle.lo_end(_G)
    print(f"rmat20 prepared in {time.time() - t0:.0f} s; max lo {lo.max()}", flush=True)
    rng = np.random.Generator(np.random.PCG64(2020))
    widest = np.argsort(-lo, kind="stable")[:16]
    classes = []
    for a, b in CLASSES:
        pool = np.nonzero((lo > a) & (lo <= b))[0]
        classes.append(rng.choice(pool, min(8, pool.size), replace=False))
    picked = np.unique(np.concatenate([widest] + classes))
    roots = {"k4": np.unique(np.concatenate([picked, np.arange(1000)])),
             "k5": np.unique(np.concatenate([picked, np.arange(100)]))}
    jobs = [(nm, int(r)) for nm in ("k5", "k4") for r in roots[nm]]
    # the widest roots first, so that the pool finishes together
    jobs.sort(key=lambda j: -int(lo[j[1]]) * (4 if j[0] == "k5" else 1))
    got = {"k4": {}, "k5": {}}
    with mp.get_context("fork").Pool(workers) as pool:
        for i, (nm, r, c) in enumerate(pool.imap_unordered(_one, jobs)):
            got[nm][r] = c
            if i % 50 == 0:
                print(f"  {i + 1}/{len(jobs)} done ({time.time() - t0:.0f} s)", flush=True)
    out = {"graph": "rmat20", "induced": True, "schedule": "analytic, Theorem 2 bounds"}
    for nm in ("k4", "k5"):
        rs = sorted(got[nm])
        out[nm] = {"roots": rs, "lo": [int(lo[r]) for r in rs], "counts": [got[nm][r] for r in rs]}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT, {nm: len(out[nm]["roots"]) for nm in ("k4", "k5")}, flush=True)


if __name__ == "__main__":
    main()
