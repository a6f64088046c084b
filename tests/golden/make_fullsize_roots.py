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

The hub stratum (above 2e6) gets a longer limit and a smaller quota: its
candidates are tried in order of increasing volume, each for up to
LIMIT_HUB_S.  `--strata 3` recomputes only that stratum and merges it into
the existing file (the other strata's roots are kept).

Run from the repository root:  python tests/golden/make_fullsize_roots.py
[--strata 0,1,2,3] (about half an hour on 8 cores for strata 0-2, up to a
few hours for the hub stratum; rewrite only when the oracle's arithmetic or
the input generators change).  `--graphs rmat22,rmat21` limits the run to
those graphs, keeping the others' stored roots."""

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
QUOTA_HUB = 6       # the hub stratum (last): roots kept,
MAX_TRIED_HUB = 16  # candidates tried (in order of increasing volume)
LIMIT_HUB_S = 240.0  # and the time limit per root
WORKERS = 8

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


def per_root_with_limit(adj, order, candidates, quota=QUOTA, limit=LIMIT_S):
    """Oracle per-root counts of the candidates, each in a forked child that
    is killed after `limit` seconds; stops once `quota` roots are kept."""
    ctx = mp.get_context("fork")
    kept, dropped, tried = [], 0, 0
    live = []  # (proc, conn, root, start)
    it = iter(candidates)
    exhausted = False
    while live or (not exhausted and len(kept) < quota):
        while not exhausted and len(live) < WORKERS and len(kept) + len(live) < quota:
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
            elif time.time() - t0 > limit:
                p.kill()
                p.join()
                a.close()
                dropped += 1
            else:
                still.append((p, a, r, t0))
        live = still
    kept.sort()
    return kept[:quota], tried, dropped


def main():
    global _G
    strata = list(range(len(STRATA)))
    if "--strata" in sys.argv:
        strata = [int(x) for x in sys.argv[sys.argv.index("--strata") + 1].split(",")]
    graphs = list(WORKLOADS)
    if "--graphs" in sys.argv:
        graphs = sys.argv[sys.argv.index("--graphs") + 1].split(",")
    old = None
    if os.path.exists(OUT) and (strata != list(range(len(STRATA))) or graphs != list(WORKLOADS)):
        with open(OUT) as f:
            old = json.load(f)
    out = {"limit_s": LIMIT_S, "quota": QUOTA, "limit_hub_s": LIMIT_HUB_S, "quota_hub": QUOTA_HUB,
           "strata": [[lo, hi if hi != float("inf") else None] for lo, hi in STRATA], "graphs": {}}
    hub = len(STRATA) - 1
    for gname, pats in WORKLOADS.items():
        if gname not in graphs:
            continue
        t0 = time.time()
        e = synth.config_graph(gname)
        _G = oracle.from_edge_tuple(e)
        del e
        deg, vol = two_hop_volume(_G)
        print(f"{gname}: prepared in {time.time() - t0:.0f} s", flush=True)
        rng = np.random.Generator(np.random.PCG64(7000 + len(gname)))
        cands = []
        for si, (lo, hi) in enumerate(STRATA):
            pool = np.nonzero((deg >= 2) & (vol > lo) & (vol <= hi))[0]
            c = rng.permutation(pool)[:MAX_TRIED]
            if si == hub:
                c = c[:MAX_TRIED_HUB]
                c = c[np.argsort(vol[c], kind="stable")]
            cands.append(c)
        gout = {}
        for nm in pats:
            adj = P.named(nm)
            order = [int(x) for x in P.pick_schedule(adj, True)[0]]
            entry = {"order": order, "roots": [], "counts": [], "stratum": [],
                     "tried": [0] * len(STRATA), "dropped": [0] * len(STRATA)}
            prev = old["graphs"][gname][nm] if old else None
            for si, c in enumerate(cands):
                if si not in strata:
                    # keep the stored stratum (strata are fixed by volume)
                    for r, v in zip(prev["roots"], prev["counts"]):
                        if STRATA[si][0] < vol[r] <= STRATA[si][1]:
                            entry["roots"].append(r)
                            entry["counts"].append(v)
                            entry["stratum"].append(si)
                    entry["tried"][si] = prev["tried"][si]
                    entry["dropped"][si] = prev["dropped"][si]
                    continue
                quota, limit = (QUOTA_HUB, LIMIT_HUB_S) if si == hub else (QUOTA, LIMIT_S)
                kept, tried, dropped = per_root_with_limit(adj, tuple(order), c, quota, limit)
                entry["roots"] += [r for r, _ in kept]
                entry["counts"] += [str(v) for _, v in kept]
                entry["stratum"] += [si] * len(kept)
                entry["tried"][si] = tried
                entry["dropped"][si] = dropped
                print(f"  {gname} {nm} stratum {si}: kept {len(kept)} of {tried} "
                      f"(dropped {dropped})", flush=True)
            gout[nm] = entry
            out["graphs"][gname] = gout
            if old:
                old = _merged(old, out, gname, gout)
            with open(OUT, "w") as f:
                json.dump(old if old else out, f, indent=1)
        _G = None
    print("wrote", OUT)


def _merged(old, out, gname, gout):
    """The old file with this graph's finished patterns replaced."""
    res = dict(old)
    for k in ("limit_s", "quota", "limit_hub_s", "quota_hub", "strata"):
        res[k] = out[k]
    res["graphs"] = {g: dict(v) for g, v in old["graphs"].items()}
    res["graphs"][gname].update(gout)
    return res


if __name__ == "__main__":
    main()
