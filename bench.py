#!/usr/bin/env python3
"""Benchmark: exact k-clique counts (K4 and K5) on an R-MAT scale-20 graph.

One step = one pass of the hot path over the resident graph: compile both
patterns (automorphisms, distinct schedules, restrictions, analytic pick,
lowering) and run both counting kernels.  Graph generation and preparation
(normalisation + degree reindex + upload) happen once before timing and are
reported separately, as the paper reports reindexing apart from mining.

Prints one JSON line.  ``value`` is the intersect throughput of the whole
step: algorithmic bytes of both patterns' bounded set operations (the same
definition as gz_count_bytes) per second of wall time.
"""

from __future__ import annotations

import argparse
import hashlib
import json
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
    "rmat20-cliques": dict(graph="rmat20", patterns=["k4", "k5"], induced=True,
                           desc="K4 and K5 counts, R-MAT scale 20, edge factor 16, "
                                "(a,b,c,d)=(0.57,0.19,0.19,0.05), seed 2001"),
    # the tailed triangle, house and K5-e of the same configuration take from
    # about 23 minutes to hours per full count, so only these two are timed
    "rmat22-induced": dict(graph="rmat22", patterns=["c4", "diamond"], induced=True,
                           desc="vertex-induced 4-cycle and diamond, R-MAT scale 22, "
                                "edge factor 16, seed 3001"),
    "er2000-triangles": dict(graph="er2000", patterns=["triangle"], induced=True,
                             desc="triangles, G(2000, 0.008), seed 1001"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in ("mine.hip",):
        with open(os.path.join(ROOT, "paper_1911_12877_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from committed rocprof counter runs
    (FETCH_SIZE + WRITE_SIZE, calibrated against a copy kernel), or None when
    absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(workload, {}).get(kernel)
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def load_valu_insts(workload, kernel):
    """VALU wave instructions per launch of `kernel` from a committed rocprof
    counter run (SQ_INSTS_VALU), or None when absent or stale."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload, {}).get(kernel)
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("valu_insts_per_launch")


def cpu_baseline(edges, pattern_names, induced, orders, bounds, target_s):
    """The oracle (single-threaded C) on a seeded sample of roots; returns
    (GB/s of algorithmic bytes, sample description)."""
    import numpy as np
    import oracle
    from oracle import patterns as P
    O = oracle.from_edge_tuple(edges)
    rng = np.random.Generator(np.random.PCG64(12345))
    n_roots = 256
    while True:
        roots = np.sort(rng.choice(O.n, size=min(n_roots, O.n), replace=False)).astype(np.int32)
        t0 = time.perf_counter()
        for nm, order, bound in zip(pattern_names, orders, bounds):
            rel = [(bound[i], i) for i in range(len(bound)) if bound[i] >= 0]
            oracle.count(O, P.named(nm), induced, order=order, relations=rel, roots=roots)
        dt = time.perf_counter() - t0
        if dt >= target_s or n_roots >= O.n:
            break
        n_roots = int(min(O.n, n_roots * max(2.0, 1.2 * target_s / max(dt, 1e-3))))
    nbytes = 0
    for nm, order, bound in zip(pattern_names, orders, bounds):
        b, _ = oracle.instrument(O, P.named(nm), induced, order, bound, roots=roots)
        nbytes += b
    desc = (f"{len(roots)} uniformly sampled roots (PCG64 seed 12345) of {O.n}, "
            f"patterns {'+'.join(pattern_names)}, same schedules and bounds")
    return nbytes / dt / 1e9, desc, dt


def learned_vs_analytic(reps=2):
    """Kernel time of the learned and the analytic schedule choice for the
    held-out patterns (6-cycle with chord {0,3} or {0,2}, K6-e, K7-e) on two
    graphs outside the model's corpus whose full counts finish in seconds:
    R-MAT scale 10 (edge factor 16, seed 8801) and Chung-Lu n = 4000
    (exponent 2.3, mean degree 10, seed 8802).  Best of `reps` timed runs per
    schedule; the counts must agree."""
    import numpy as np
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20-cliques", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned vs analytic schedule comparison")
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

    import numpy as np
    import torch
    from paper_1911_12877_amd import gz, motifs, synth

    wl = WORKLOADS[args.workload]
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
    log(f"prepared graph n={info['n']} nnz={info['nnz']} max_deg={info['max_deg']} "
        f"max_lo={info['max_lo_deg']} in {t_prep:.2f}s")

    adjs = [motifs.named(nm) for nm in wl["patterns"]]
    scheds = [gz.compile_pattern(a, wl["induced"]) for a in adjs]
    infos = [s.info() for s in scheds]
    alg_bytes = []
    counts = []
    for nm, s in zip(wl["patterns"], scheds):
        if args.no_alg_bytes:
            c, _ = gz.count_timed(G, s, stream=stream)
            b = None
        else:
            b, c = gz.count_bytes(G, s, stream=stream)
        alg_bytes.append(b)
        counts.append(c)
        log(f"{nm}: count={c} algorithmic bytes={b}")

    def step():
        ks = []
        for nm, a in zip(wl["patterns"], adjs):
            s = gz.compile_pattern(a, wl["induced"])
            c, ms = gz.count_timed(G, s, stream=stream)
            ks.append((c, ms))
        return ks

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kern_ms = [0.0] * len(adjs)
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = step()
        for j, (c, ms) in enumerate(res):
            assert c == counts[j], "count changed between runs"
            kern_ms[j] += ms
        log(f"step {i}: " + ", ".join(f"{nm} {ms:.2f} ms" for nm, (_, ms) in
                                      zip(wl["patterns"], res)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    avg_ms = [m / args.steps for m in kern_ms]
    have_bytes = all(b is not None for b in alg_bytes)
    value = sum(alg_bytes) / (ms_per_step / 1e3) / 1e9 if have_bytes else None

    dom = int(np.argmax(avg_ms))
    kdom = len(adjs[dom])
    traffic = load_traffic(args.workload, wl["patterns"][dom])
    ops = None
    try:  # clique schedules run on bit rows: an ALU-bound kernel pair
        ops, _ = gz.count_ops(G, scheds[dom], stream=stream)
    except gz.GzError:
        ops = None
    if ops is not None:
        achieved = ops / (avg_ms[dom] / 1e3) / 1e9
        valu = load_valu_insts(args.workload, wl["patterns"][dom])
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": ALU_PEAK_GOPS,
                    "unit": "Gop/s", "frac": round(achieved / ALU_PEAK_GOPS, 4),
                    "traffic": traffic, "ops_per_launch": ops,
                    "valu_issue_frac": (round(valu / (avg_ms[dom] / 1e3) / VALU_ISSUE_PEAK, 4)
                                        if valu else None),
                    "kernel": f"k_clique_wave<{kdom}> + k_clique_block<{kdom}>",
                    "pattern": wl["patterns"][dom], "kernel_ms": round(avg_ms[dom], 4)}
    else:
        achieved = alg_bytes[dom] / (avg_ms[dom] / 1e3) / 1e9 if have_bytes else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 2) if have_bytes else None,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4) if have_bytes else None,
                    "traffic": traffic, "kernel": f"k_mine<{kdom}>",
                    "pattern": wl["patterns"][dom], "kernel_ms": round(avg_ms[dom], 4)}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a root sample ...")
        gbs, desc, dt = cpu_baseline(edges, wl["patterns"], wl["induced"],
                                     [i["order"] for i in infos], [i["bound"] for i in infos],
                                     args.cpu_seconds)
        cpu = {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": desc, "seconds": round(dt, 2)}

    lva = None if args.no_learned else learned_vs_analytic()

    out = {
        "metric": METRIC, "value": round(value, 2) if have_bytes else None, "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "graph": wl["desc"], "n": info["n"],
                   "nnz": info["nnz"], "patterns": wl["patterns"],
                   "induced": wl["induced"], "schedule": "analytic",
                   "parallelism": "single GPU"},
        "counts": {nm: c for nm, c in zip(wl["patterns"], counts)},
        "kernel_ms": {nm: round(m, 4) for nm, m in zip(wl["patterns"], avg_ms)},
        "alg_bytes": {nm: b for nm, b in zip(wl["patterns"], alg_bytes)},
        "counts_per_s": round(sum(counts) / (ms_per_step / 1e3), 1),
        "prep_s": round(t_prep, 3),
        "prep_device_s": round(t_prep_dev, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned_vs_analytic": lva,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
