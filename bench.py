#!/usr/bin/env python3
"""Benchmark: exact vertex-induced pattern counts on one MI355X.

Default workload (``rmat22-induced``): the vertex-induced 4-cycle, diamond and
tailed triangle on an R-MAT scale-22 graph (edge factor 16,
(a,b,c,d) = (0.57,0.19,0.19,0.05), seed 3001; 4,194,304 vertices, 128.3 M
neighbour entries), each with the analytic model's schedule, its symmetry
restrictions and the degree orientation.  The count of a pattern decomposes
exactly over the roots of its first loop (every instance has one restricted
mapping), so the job is cut into S strided root slices (roots r with
r = q mod S): one step counts every pattern of the workload over one slice,
and S consecutive steps are one complete exact count of every pattern.
Slices hold equal shares of every degree range, so their times agree to
about 1%.  The full-count time of a pattern is the sum over one cycle of
slices; it is reported whenever the timed steps cover a cycle.

Other workloads: ``rmat20-cliques`` (K4 and K5 on R-MAT scale 20, one full
count of each per step), ``er2000-triangles`` (triangles of G(2000, 0.008))
and ``census64-motif4`` (the six connected 4-vertex induced patterns over the
64 Chung-Lu graphs of the motif batch, one replay of the captured census
launch per step).

The learned-schedule comparison runs the held-out patterns (6-cycle with a
chord, K6-e, K7-e) with the analytic and the learned choice on two small
graphs in full, and with --learned-large on the learned-schedule workload's
R-MAT 21 and Chung-Lu 2M graphs over a seeded sample of low-volume roots.

Graph generation and preparation (normalisation, degree reindex, upload)
happen once before timing and are reported apart, as the paper reports its
reindexing apart from mining.  Every step compiles its patterns (Aut,
Algorithm 3, Algorithm 1 with Theorem 2, analytic pick, lowering) and runs the
counts on the resident graph.

Prints one JSON line.  ``value`` is exact instances counted per second of
wall time over the timed steps.  ``roofline`` is the dominant kernel's rate
against its bound; ``cpu_baseline`` is the oracle (plain C, one process per
core, roots sharded) on a seeded root sample, in the same unit.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact-count wall time & intersect GB/s, learned vs analytic schedule, 1 GPU"
HBM_PEAK_GBS = 8000.0
# 32-bit integer VALU: 256 CUs x 64 lanes per clock x 2.4 GHz (the FP32
# vector figure of 157.3 TFLOP/s counts packed pairs and FMA as two each)
ALU_PEAK_GOPS = 256 * 64 * 2.4
# wave64 VALU instructions issued per second: one per CU per clock
VALU_ISSUE_PEAK = 256 * 2.4e9

WORKLOADS = {
    # the house (and K5-e) of the same configuration are far beyond a
    # benchmark run with this method: see the design notes
    "rmat22-induced": dict(graph="rmat22", patterns=["c4", "diamond", "tailed_triangle"],
                           induced=True, slices=128,
                           desc="vertex-induced 4-cycle, diamond and tailed triangle, R-MAT "
                                "scale 22, edge factor 16, (a,b,c,d)=(0.57,0.19,0.19,0.05), "
                                "seed 3001"),
    "rmat20-cliques": dict(graph="rmat20", patterns=["k4", "k5"], induced=True, slices=1,
                           desc="K4 and K5 counts, R-MAT scale 20, edge factor 16, "
                                "(a,b,c,d)=(0.57,0.19,0.19,0.05), seed 2001"),
    "er2000-triangles": dict(graph="er2000", patterns=["triangle"], induced=True, slices=1,
                             desc="triangles, G(2000, 0.008), seed 1001"),
    # the 21 five-vertex patterns of the same batch are out of reach for the
    # largest graphs (the 5-star alone enumerates ~4e14 leaf sets)
    "census64-motif4": dict(graph="census64", patterns=["motif4"], induced=True, slices=1,
                            desc="census of the 6 connected 4-vertex induced patterns over the "
                                 "64 Chung-Lu graphs of the motif batch (seeds 4001..4064), "
                                 "one captured launch"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in ("mine.hip",):
        with open(os.path.join(ROOT, "paper_1911_12877_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(workload, pattern):
    """Per-launch counter figures of `pattern`'s kernel from a committed
    rocprof run (HBM bytes from FETCH_SIZE + WRITE_SIZE calibrated against a
    copy kernel, VALU instructions), or {} when absent or taken on a
    different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f).get(workload, {}).get(pattern)
    if not rec or rec.get("source_hash") != source_hash():
        return {}
    return rec


# ------------------------------------------------------------ CPU baseline

_CPU = {}  # prepared graph and schedules, inherited by forked workers


def _cpu_shard(roots):
    import oracle
    from oracle import patterns as P
    O = _CPU["graph"]
    t0 = time.perf_counter()
    total = 0
    for nm, order, bound in _CPU["scheds"]:
        rel = [(bound[i], i) for i in range(len(bound)) if bound[i] >= 0]
        total += oracle.count(O, P.named(nm), _CPU["induced"], order=order, relations=rel,
                              roots=roots)
    return total, time.perf_counter() - t0


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(edges, pattern_names, induced, orders, bounds, target_s, workers):
    """The oracle (single-threaded C per process) on a seeded uniform sample
    of roots, the same schedules and bounds as the GPU; the sample grows
    until one core needs about target_s.  Then the same sample sharded
    round-robin over `workers` processes.  Returns instances/s of both."""
    import numpy as np
    import oracle
    _CPU["graph"] = oracle.from_edge_tuple(edges)
    _CPU["scheds"] = list(zip(pattern_names, orders, bounds))
    _CPU["induced"] = induced
    n = _CPU["graph"].n
    rng = np.random.Generator(np.random.PCG64(12345))
    perm = rng.permutation(n).astype(np.int32)
    n_roots = 256
    while True:
        roots = np.sort(perm[:min(n_roots, n)])
        count1, dt1 = _cpu_shard(roots)
        if dt1 >= target_s or n_roots >= n:
            break
        n_roots = int(min(n, n_roots * max(2.0, 1.2 * target_s / max(dt1, 1e-3))))
    shards = [roots[w::workers] for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_cpu_shard, shards)
    dtn = time.perf_counter() - t0
    countn = sum(c for c, _ in res)
    assert countn == count1, "sharded oracle disagrees with the single-process run"
    _CPU.clear()
    desc = (f"{len(roots)} uniformly sampled roots (PCG64 seed 12345) of {n}, "
            f"patterns {'+'.join(pattern_names)}, same schedules and bounds")
    return count1 / dt1, dt1, countn / dtn, dtn, desc


# --------------------------------------------------------- learned schedules


def learned_vs_analytic(reps=2):
    """Kernel time of the learned and the analytic schedule choice for the
    held-out patterns (6-cycle with chord {0,3} or {0,2}, K6-e, K7-e) on two
    graphs outside the model's corpus whose full counts finish in seconds:
    R-MAT scale 10 (edge factor 16, seed 8801) and Chung-Lu n = 4000
    (exponent 2.3, mean degree 10, seed 8802).  Best of `reps` timed runs per
    schedule; the counts must agree."""
    from paper_1911_12877_amd import gz, learn, synth
    if not os.path.exists(learn.MODEL_PATH):
        return None
    learn.install()
    cases = []
    ta = tl = 0.0
    same = True
    for gname, e in (("rmat10", synth.rmat_edges(10, 16, seed=8801)),
                     ("cl4000", synth.chung_lu_edges(4000, 2.3, 10.0, 8802, cap=True))):
        G = gz.load_edges(*e)
        for nm, a in learn.held_out_patterns().items():
            sa = gz.compile_pattern(a, True)
            sl = gz.compile_pattern_graph(G, a, True, gz.SCHED_LEARNED)
            ca, ma = learn.time_schedule(G, sa, reps=reps)
            cl, ml = learn.time_schedule(G, sl, reps=reps)
            same = same and ca == cl
            ta += ma
            tl += ml
            cases.append({"graph": gname, "pattern": nm, "analytic_ms": round(ma, 3),
                          "learned_ms": round(ml, 3)})
            log(f"learned vs analytic {gname} {nm}: {ma:.2f} ms -> {ml:.2f} ms")
    return {"analytic_ms": round(ta, 3), "learned_ms": round(tl, 3),
            "speedup": round(ta / tl, 3) if tl > 0 else None, "counts_equal": same,
            "cases": cases}


def learned_vs_analytic_cfg5(per_stratum=(256, 32), bounds=(1e4, 2e4)):
    """Learned and analytic schedule choices for the held-out patterns on the
    learned-schedule workload's own graphs, R-MAT scale 21 (seed 5001) and
    Chung-Lu n = 2M (exponent 2.2, mean degree 16, seed 5002), over one
    seeded root sample per graph, the same for both choices: roots of
    two-hop volume (sum of neighbour degrees) up to 1e4 and in (1e4, 2e4].
    Heavier roots take 10-90 s each for the 6-cycle with a chord under a
    good schedule and far longer under a poor one, so full counts and the
    upper strata are out of reach here; this is a sample."""
    import numpy as np
    from paper_1911_12877_amd import gz, learn, synth
    if not os.path.exists(learn.MODEL_PATH):
        return None
    learn.install()
    cases = []
    for gname in ("rmat21", "cl2m"):
        e = synth.config_graph(gname)
        G = gz.load_edges(*e, flags=gz.GRAPH_PREP_DEVICE)
        del e
        r, c, _ = gz.graph_export(G)
        deg = np.diff(r).astype(np.int64)
        cs = np.concatenate([[0], np.cumsum(deg[c])])
        vol = cs[r[1:].astype(np.int64)] - cs[r[:-1].astype(np.int64)]
        del c, cs
        rng = np.random.Generator(np.random.PCG64(5150))
        roots = []
        for k, (lo, hi) in zip(per_stratum, ((0, bounds[0]), (bounds[0], bounds[1]))):
            pool = np.nonzero((deg >= 2) & (vol > lo) & (vol <= hi))[0]
            roots.append(rng.choice(pool, min(k, pool.size), replace=False))
        roots = np.sort(np.concatenate(roots)).astype(np.int32)
        for nm, a in learn.held_out_patterns().items():
            sa = gz.compile_pattern(a, True)
            sl = gz.compile_pattern_graph(G, a, True, gz.SCHED_LEARNED)
            log(f"learned vs analytic {gname} {nm}: analytic ...")
            ca, ma = gz.count_subset(G, sa, roots)
            if sl.info()["order"] == sa.info()["order"]:
                cl, ml = ca, ma  # the same schedule (e.g. a graph outside the corpus's range)
            else:
                log(f"learned vs analytic {gname} {nm}: learned ...")
                cl, ml = gz.count_subset(G, sl, roots)
            cases.append({"graph": gname, "pattern": nm, "roots": int(roots.size),
                          "analytic_ms": round(ma, 3), "learned_ms": round(ml, 3),
                          "same_schedule": sa.info()["order"] == sl.info()["order"],
                          "counts_equal": ca == cl})
            log(f"learned vs analytic {gname} {nm} ({roots.size} roots): "
                f"{ma:.2f} ms -> {ml:.2f} ms")
        del G
    ta = sum(c["analytic_ms"] for c in cases)
    tl = sum(c["learned_ms"] for c in cases)
    return {"analytic_ms": round(ta, 3), "learned_ms": round(tl, 3),
            "speedup": round(ta / tl, 3) if tl > 0 else None,
            "counts_equal": all(c["counts_equal"] for c in cases),
            "sample": f"seeded roots of two-hop volume <= {bounds[0]:.0e} ({per_stratum[0]}) "
                      f"and in ({bounds[0]:.0e}, {bounds[1]:.0e}] ({per_stratum[1]}) per graph",
            "cases": cases}


def census_main(args, wl):
    """The motif-census workload: one step replays the captured census
    launch over all (graph, pattern) pairs."""
    import numpy as np
    import torch
    from paper_1911_12877_amd import gz, motifs, synth
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    params = [synth.census_graph_params(i) for i in range(64)]
    graphs = [gz.load_edges(*synth.config_graph(p), flags=gz.GRAPH_PREP_DEVICE) for p in params]
    t_prep = time.perf_counter() - t0
    pats = motifs.connected_patterns(4)
    scheds = [gz.compile_pattern(a, True) for a in pats]
    census = gz.Census(graphs, scheds)
    log(f"64 graphs prepared in {t_prep:.1f}s; {len(pats)} patterns")
    ref = None
    for i in range(args.warmup):
        ref, ms = census.run()
        log(f"warmup {i}: {ms:.1f} ms")
    kern = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        counts, ms = census.run()
        if ref is not None:
            assert np.array_equal(counts, ref), "census counts changed between replays"
        ref = counts
        kern.append(ms)
        log(f"step {i}: {ms:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total = int(ref.astype(object).sum())
    alg = None
    if not args.no_alg_bytes:
        # the census runs the same loops as single counts: their bytes
        alg = sum(gz.count_bytes(G, s)[0] for G in graphs for s in scheds)
    km = float(np.mean(kern))
    achieved = alg / (km / 1e3) / 1e9 if alg else None
    out = {
        "metric": METRIC, "value": round(total * args.steps / wall, 1), "unit": "instances/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": True,
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "graph": wl["desc"], "graphs": 64,
                   "patterns": len(pats), "induced": True, "schedule": "analytic",
                   "step": "one replay of the captured census launch",
                   "parallelism": "single GPU"},
        "census_total": total, "prep_s": round(t_prep, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2) if alg else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if alg else None,
                     "traffic": None, "alg_bytes_per_launch": alg,
                     "kernel": "k_census<5>", "kernel_ms": round(km, 3)},
        "cpu_baseline": None, "learned_vs_analytic": None,
    }
    print(json.dumps(out), flush=True)


def copy_calibration():
    """A plain copy kernel of known size: 5 copies of 1 GiB (2^28 int32)
    device to device; each moves 1 GiB in and 1 GiB out of HBM."""
    import torch
    torch.cuda.set_device(0)
    x = torch.arange(1 << 28, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    assert int(y[-1].item()) == (1 << 28) - 1
    print(json.dumps({"copy_bytes_per_launch": 1 << 30, "launches": 5}), flush=True)


# -------------------------------------------------------------------- main


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22-induced", choices=sorted(WORKLOADS))
    ap.add_argument("--slices", type=int, default=None,
                    help="root slices per complete count (default: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned vs analytic schedule comparison")
    ap.add_argument("--learned-large", action="store_true",
                    help="also compare the two schedule choices on the R-MAT 21 and "
                         "Chung-Lu 2M graphs over a low-volume root sample (minutes)")
    ap.add_argument("--no-alg-bytes", action="store_true",
                    help="skip the instrumented pass (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 5 times "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the count shards by root; see the design notes)", file=sys.stderr)
        sys.exit(2)

    wl = WORKLOADS[args.workload]
    if wl["graph"] == "census64":
        census_main(args, wl)
        return

    import numpy as np
    import torch
    from paper_1911_12877_amd import gz, motifs, synth

    S = max(1, args.slices or wl["slices"])
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    t0 = time.perf_counter()
    edges = synth.config_graph(wl["graph"])
    t_gen = time.perf_counter() - t0
    log(f"generated {wl['graph']}: {edges[0].shape[0]} samples in {t_gen:.1f}s")
    t0 = time.perf_counter()
    G = gz.load_edges(*edges, stream=stream)
    t_prep = time.perf_counter() - t0
    # the same preparation on the device (radix sorts); identical arrays
    t0 = time.perf_counter()
    Gd = gz.load_edges(*edges, flags=gz.GRAPH_PREP_DEVICE, stream=stream)
    t_prep_dev = time.perf_counter() - t0
    assert Gd.info() == G.info()
    del Gd
    info = G.info()
    n = info["n"]
    log(f"prepared graph n={n} nnz={info['nnz']} max_deg={info['max_deg']} "
        f"max_lo={info['max_lo_deg']} in {t_prep:.2f}s")

    pats = wl["patterns"]
    adjs = [motifs.named(nm) for nm in pats]
    infos = [gz.compile_pattern(a, wl["induced"]).info() for a in adjs]
    all_roots = np.arange(n, dtype=np.int32)
    slices = [all_roots[q::S] for q in range(S)]

    def step(i):
        """Compile and count every pattern over slice i mod S (the whole
        graph when S == 1): [(count, kernel ms)] per pattern."""
        q = i % S
        out = []
        for a in adjs:
            s = gz.compile_pattern(a, wl["induced"])
            if S == 1:
                out.append(gz.count_timed(G, s, stream=stream))
            else:
                out.append(gz.count_subset(G, s, slices[q], stream=stream))
        return q, out

    for i in range(args.warmup):
        q, res = step(i)
        log(f"warmup {i} (slice {q}): " + ", ".join(f"{nm} {ms:.1f} ms" for nm, (_, ms) in
                                                      zip(pats, res)))
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        q, res = step(i)
        recs.append((q, res))
        log(f"step {i - args.warmup} (slice {q}): " +
            ", ".join(f"{nm} {c} in {ms:.1f} ms" for nm, (c, ms) in zip(pats, res)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    total_count = sum(c for _, res in recs for c, _ in res)
    value = total_count / wall

    # per pattern over the timed steps; complete counts when a cycle of
    # slices was covered (the first S timed steps: S consecutive residues)
    kern_ms = [sum(res[j][1] for _, res in recs) for j in range(len(pats))]
    per_pattern = {}
    for j, nm in enumerate(pats):
        d = {"kernel_ms_per_step": round(kern_ms[j] / args.steps, 3),
             "order": list(infos[j]["order"]), "bound": infos[j]["bound"]}
        if args.steps >= S:
            cyc = recs[:S]
            d["count"] = sum(res[j][0] for _, res in cyc)
            d["full_count_kernel_s"] = round(sum(res[j][1] for _, res in cyc) / 1e3, 3)
        per_pattern[nm] = d

    # dominant kernel: the pattern with the largest kernel time per step
    dom = int(np.argmax(kern_ms))
    dname = pats[dom]
    kdom = len(adjs[dom])
    ctr = load_counters(args.workload, dname)
    sdom = gz.compile_pattern(adjs[dom], wl["induced"])
    ops = None
    try:  # clique schedules run on bit rows: an ALU-bound kernel pair
        ops, _ = gz.count_ops(G, sdom, stream=stream) if S == 1 else (None, None)
    except gz.GzError:
        ops = None
    q_dom = recs[0][0]
    ms_dom = np.mean([res[dom][1] for q, res in recs if q == q_dom])
    if ops is not None:
        achieved = ops / (ms_dom / 1e3) / 1e9
        valu = ctr.get("valu_insts_per_launch")
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": ALU_PEAK_GOPS,
                    "unit": "Gop/s", "frac": round(achieved / ALU_PEAK_GOPS, 4),
                    "traffic": ctr.get("bytes_per_launch"), "ops_per_launch": ops,
                    "valu_issue_frac": (round(valu / (ms_dom / 1e3) / VALU_ISSUE_PEAK, 4)
                                        if valu else None),
                    "kernel": f"k_clique_wave<{kdom}> + k_clique_block<{kdom}>",
                    "pattern": dname, "kernel_ms": round(float(ms_dom), 4)}
    else:
        alg = None
        if not args.no_alg_bytes:
            # algorithmic bytes of the same launch: one instrumented pass
            # over the dominant pattern's first timed slice
            if S == 1:
                alg, _ = gz.count_bytes(G, sdom, stream=stream)
            else:
                alg, _ = gz.count_bytes_subset(G, sdom, slices[q_dom], stream=stream)
        achieved = alg / (ms_dom / 1e3) / 1e9 if alg is not None else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 2) if alg else None,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4) if alg else None,
                    "traffic": ctr.get("bytes_per_launch"), "alg_bytes_per_launch": alg,
                    "valu_issue_frac": (round(ctr["valu_insts_per_launch"] / (ms_dom / 1e3) /
                                              VALU_ISSUE_PEAK, 4)
                                        if ctr.get("valu_insts_per_launch") else None),
                    "kernel": f"k_mine<{kdom}>", "pattern": dname,
                    "launch": f"slice {q_dom} of {S}" if S > 1 else "full count",
                    "kernel_ms": round(float(ms_dom), 4)}

    cpu = None
    if not args.no_cpu_baseline:
        workers = cpu_cores()
        log(f"timing the oracle on a root sample (1 core, then {workers}) ...")
        v1, dt1, vn, dtn, desc = cpu_baseline(
            edges, pats, wl["induced"], [i["order"] for i in infos], [i["bound"] for i in infos],
            args.cpu_seconds, workers)
        cpu = {"value": round(vn, 1), "unit": "instances/s", "cores": workers, "kind": "oracle",
               "sample": desc, "seconds": round(dtn, 2),
               "one_core": {"value": round(v1, 1), "seconds": round(dt1, 2)}}

    lva = None if args.no_learned else learned_vs_analytic()
    lva5 = learned_vs_analytic_cfg5() if args.learned_large else None

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "instances/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "graph": wl["desc"], "n": n,
                   "nnz": info["nnz"], "patterns": pats, "induced": wl["induced"],
                   "schedule": "analytic",
                   "step": (f"every pattern over one of {S} strided root slices"
                            if S > 1 else "one full count of every pattern"),
                   "parallelism": "single GPU"},
        "patterns": per_pattern,
        "prep_s": round(t_prep, 3),
        "prep_device_s": round(t_prep_dev, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned_vs_analytic": lva,
        "learned_vs_analytic_rmat21_cl2m": lva5,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
