"""Writes fullsize_roots.json: per-root counts at the full-size workloads,
computed by the oracle alone, for the GPU parity tests to compare against.

Workloads: vertex-induced 4-cycle, diamond, tailed triangle, house and K5-e
on R-MAT scale 22; vertex-induced 6-cycle with a chord ({0,3} or {0,2}),
K6-e and K7-e on R-MAT scale 21 and on the Chung-Lu graph of 2M vertices.
Schedule: the analytic model's pick (Section 5.1 cost in G(n=1000, p=5/999),
Algorithm 3's distinct schedules) with Theorem 2's single bound per loop;
a per-root count is the number of instances whose restricted mapping puts
that root in the first loop, so the counts decompose the total exactly.

Roots are drawn, seeded, from four strata of two-hop volume
vol(v) = sum of deg(u) over u in N(v) (vertices of degree >= 2):
(0, 2e4], (2e4, 2e5], (2e5, 2e6] and above 2e6.  A full count of these
graphs is far beyond the oracle, and so is a single hub root of a heavy
pattern, so each candidate root runs in a child process under a time limit;
roots that finish within it are kept until the stratum's quota is filled.
The file records, per stratum, how many candidates were tried and dropped.

Run from the repository root:  python tests/golden/make_fullsize_roots.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_roots.json")
WORKLOADS = {
    "rmat22": ["c4", "diamond", "tailed_triangle", "house", "k5e"],
    "rmat21": ["c6chord03", "c6chord02", "k6e", "k7e"],
    "cl2m": ["c6chord03", "c6chord02", "k6e", "k7e"],
}
STRATA = [(0.0, 2e4), (2e4, 2e5), (2e5, 2e6), (2e6, float("inf"))]
QUOTA = 12          # roots kept per stratum
MAX_TRIED = 48      # candidates tried per stratum
LIMIT_S = 3.0       # oracle time limit per root
WORKERS = 6

_G = None  # the prepared graph, inherited by forked children


def two_hop_volume(g):
    deg = np.diff(g.rowptr).astype(np.int64)
    cs = np.concatenate([[0], np.cumsum(deg[g.col])])
    rp = g.rowptr.astype(np.int64)
    return deg, cs[rp[1:]] - cs[rp[:-1]]


def _child(conn, adj, order, root):
    _, per = oracle.count(_G, adj, True, order=order, relations="thm2",
                          roots=np.array([root], np.int32), per_root=True)
    conn.send(int(per[0]))
    conn.close()


def per_root_with_limit(adj, order, candidates):
    """Oracle per-root counts of the candidates, each in a forked child that
    is killed after LIMIT_S; stops once QUOTA roots are kept."""
    ctx = mp.get_context("fork")
    kept, dropped, tried = [], 0, 0
    live = []  # (proc, conn, root, start)
    it = iter(candidates)
    exhausted = False
    while live or (not exhausted and len(kept) < QUOTA):
        while not exhausted and len(live) < WORKERS and len(kept) + len(live) < QUOTA:
            try:
                r = int(next(it))
            except StopIteration:
                exhausted = True
                break
            a, b = ctx.Pipe(duplex=False)
            p = ctx.Process(target=_child, args=(b, adj, order, r))
            p.start()
            b.close()
            live.append((p, a, r, time.time()))
            tried += 1
        time.sleep(0.02)
        still = []
        for p, a, r, t0 in live:
            if a.poll():
                kept.append((r, a.recv()))
                p.join()
                a.close()
            elif time.time() - t0 > LIMIT_S:
                p.kill()
                p.join()
                a.close()
                dropped += 1
            else:
                still.append((p, a, r, t0))
        live = still
    kept.sort()
    return kept[:QUOTA], tried, dropped


def main():
    global _G
    out = {"limit_s": LIMIT_S, "quota": QUOTA, "strata": [[lo, hi if hi != float("inf") else None]
                                                          for lo, hi in STRATA], "graphs": {}}
    for gname, pats in WORKLOADS.items():
        t0 = time.time()
        e = synth.config_graph(gname)
        _G = oracle.from_edge_tuple(e)
        del e
        deg, vol = two_hop_volume(_G)
        print(f"{gname}: prepared in {time.time() - t0:.0f} s", flush=True)
        rng = np.random.Generator(np.random.PCG64(7000 + len(gname)))
        cands = []
        for lo, hi in STRATA:
            pool = np.nonzero((deg >= 2) & (vol > lo) & (vol <= hi))[0]
            cands.append(rng.permutation(pool)[:MAX_TRIED])
        gout = {}
        for nm in pats:
            adj = P.named(nm)
            order = [int(x) for x in P.pick_schedule(adj, True)[0]]
            entry = {"order": order, "roots": [], "counts": [], "tried": [], "dropped": []}
            for si, c in enumerate(cands):
                kept, tried, dropped = per_root_with_limit(adj, tuple(order), c)
                entry["roots"] += [r for r, _ in kept]
                entry["counts"] += [str(v) for _, v in kept]
                entry["tried"].append(tried)
                entry["dropped"].append(dropped)
                print(f"  {gname} {nm} stratum {si}: kept {len(kept)} of {tried} "
                      f"(dropped {dropped})", flush=True)
            gout[nm] = entry
        out["graphs"][gname] = gout
        _G = None
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
