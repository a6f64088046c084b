"""Learned schedule cost model: corpus collection, training and the bundled
weights.

The corpus is the compiler's own output: every distinct schedule
(Algorithm 3) of a set of training patterns, each counted on a set of small
synthetic training graphs, with its kernel time measured.  Targets are
log10 run times centred within each (pattern, graph) group, so the model
learns a ranking of schedules rather than the absolute cost of a graph.
Training runs on the GPU through libgz's MLP kernels (FP32 forward,
backward and Adam); ranking at compile time uses BF16 inference.  The
patterns whose schedules the model is evaluated on (the 6-cycle with one
chord, K6 minus an edge, K7 minus an edge) are never in the corpus.

A learned choice replaces the analytic model's pick only when the network
predicts it faster by more than twice its validation error (group-wise
cross-validation over the corpus, stored with the weights as `margin`), only
for patterns no larger than the corpus's (`k_max`), and only on graphs whose
statistics lie within the corpus's range (`graph_min`, `graph_max`): the
network was never trained beyond them.

Command line (GPU):  python -m paper_1911_12877_amd.learn collect OUT.npz
                     python -m paper_1911_12877_amd.learn train IN.npz [MODEL.npz]
                     python -m paper_1911_12877_amd.learn margin IN.npz [MODEL.npz]
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

from . import gz, motifs, synth

H_DEFAULT = 128
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models",
                          "cost_mlp.npz")


# ------------------------------------------------------------- patterns

def _edges_adj(k, edges):
    a = np.zeros((k, k), dtype=np.uint8)
    for u, v in edges:
        a[u, v] = a[v, u] = 1
    return a


def _connected(a):
    k = a.shape[0]
    seen, stack = {0}, [0]
    while stack:
        v = stack.pop()
        for u in np.nonzero(a[v])[0]:
            if int(u) not in seen:
                seen.add(int(u))
                stack.append(int(u))
    return len(seen) == k


def canonical(a):
    """Canonical code of a pattern (largest upper-triangle bit string over
    all relabellings), as the census computes it."""
    return motifs.canonical_code(a)


def held_out_patterns():
    c6 = [(i, (i + 1) % 6) for i in range(6)]
    k6e = [(i, j) for i in range(6) for j in range(i + 1, 6) if (i, j) != (4, 5)]
    k7e = [(i, j) for i in range(7) for j in range(i + 1, 7) if (i, j) != (5, 6)]
    return {
        "c6chord03": _edges_adj(6, c6 + [(0, 3)]),
        "c6chord02": _edges_adj(6, c6 + [(0, 2)]),
        "k6e": _edges_adj(6, k6e),
        "k7e": _edges_adj(7, k7e),
    }


def connected_patterns(k):
    """The connected k-vertex patterns in canonical-code order (the corpus's
    order)."""
    return sorted(motifs.connected_patterns(k), key=motifs.canonical_code)


def random_patterns(k, count, seed, exclude_codes, min_edges=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = [(i, j) for i in range(k) for j in range(i + 1, k)]
    out, codes = [], set(exclude_codes)
    while len(out) < count:
        keep = rng.random(len(pairs)) < rng.uniform(0.3, 0.8)
        a = _edges_adj(k, [p for p, kk in zip(pairs, keep) if kk])
        if int(a.sum()) // 2 < min_edges or not _connected(a):
            continue
        c = canonical(a)
        if c in codes:
            continue
        codes.add(c)
        out.append(a)
    return out


def training_patterns():
    held = {canonical(a) for a in held_out_patterns().values()}
    pats = [a for k in (3, 4, 5) for a in connected_patterns(k) if canonical(a) not in held]
    # sparse 6-vertex patterns have huge induced counts on power-law graphs;
    # the corpus keeps the denser ones (at least 8 of 15 edges)
    big = random_patterns(6, 20, 606, held, min_edges=8)
    return pats, big


def training_graphs():
    """(name, edge list, small) - `small` graphs also get the 6-vertex
    patterns."""
    return [
        ("rmat9a", synth.rmat_edges(9, 8, seed=3101), True),
        ("cl1500", synth.chung_lu_edges(1500, 2.3, 6.0, 3102, cap=True), True),
        ("er1000", synth.er_edges(1000, 0.006, 3103), True),
        ("rmat10b", synth.rmat_edges(10, 12, seed=3104), False),
        ("cl5000", synth.chung_lu_edges(5000, 2.6, 12.0, 3105, cap=True), False),
        ("rmat11c", synth.rmat_edges(11, 6, abcd=(0.45, 0.22, 0.22, 0.11), seed=3106), False),
    ]


# ------------------------------------------------------------ collection

def time_schedule(G, sched, reps=2, repeat_below_ms=50.0):
    """(count, fastest kernel ms); runs taking longer than repeat_below_ms
    are not repeated."""
    best = None
    count = None
    for _ in range(reps):
        c, ms = gz.count_timed(G, sched)
        count = c
        best = ms if best is None else min(best, ms)
        if ms > repeat_below_ms:
            break
    return count, best


def collect(out_path, max_sched_big=8, log=print):
    pats, big = training_patterns()
    X, y, grp, meta = [], [], [], []
    gid = 0
    for gname, e, small in training_graphs():
        G = gz.load_edges(*e)
        plist = [(a, True) for a in pats] + ([(a, True) for a in big] if small else [])
        t0 = time.time()
        for a, induced in plist:
            scheds = gz.enumerate_schedules(a, induced)
            if a.shape[0] >= 6 and len(scheds) > max_sched_big:
                rng = np.random.Generator(np.random.PCG64(gid))
                pick = sorted(rng.choice(len(scheds), max_sched_big, replace=False))
                an = gz.compile_pattern(a, induced).info()["order"]
                idx = [i for i, (o, _) in enumerate(scheds) if o == an]
                scheds = [scheds[i] for i in sorted(set(pick) | set(idx))]
            rows = []
            counts = set()
            for order, _ in scheds:
                s = gz.compile_pattern_order(a, order, induced)
                c, ms = time_schedule(G, s)
                counts.add(c)
                rows.append((gz.schedule_features(G, a, order, induced), np.log10(max(ms, 1e-3))))
            assert len(counts) == 1, "schedules disagree on the count"
            slowest = max(10 ** t for _, t in rows)
            log(f"  {gname} k={a.shape[0]} code={canonical(a)} schedules={len(rows)} "
                f"slowest={slowest:.1f} ms", flush=True)
            for f, t in rows:
                X.append(f)
                y.append(t)
                grp.append(gid)
            meta.append((gname, canonical(a), len(rows)))
            gid += 1
        log(f"collected {gname}: {len(plist)} patterns, {len(y)} rows so far, "
            f"{time.time() - t0:.1f}s", flush=True)
        np.savez(out_path, X=np.array(X, dtype=np.float32), y=np.array(y, dtype=np.float64),
                 group=np.array(grp, dtype=np.int32))
    X = np.array(X, dtype=np.float32)
    y = np.array(y, dtype=np.float64)
    grp = np.array(grp, dtype=np.int32)
    np.savez(out_path, X=X, y=y, group=grp)
    return X, y, grp


def centred(y, grp, clip=1.0):
    """Training targets: log10 times clipped at `clip` decades above the
    group's fastest schedule (the ranking only needs the near-best ones
    right), then centred within each group."""
    yc = np.array(y, dtype=np.float64).copy()
    for g in np.unique(grp):
        m = grp == g
        if clip is not None:
            yc[m] = np.minimum(yc[m], yc[m].min() + clip)
        yc[m] -= yc[m].mean()
    return yc


# -------------------------------------------------------------- training

def init_params(D, H, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.uniform(-1, 1, (H, D)) * np.sqrt(6.0 / D)
    w2 = rng.uniform(-1, 1, H) * np.sqrt(6.0 / H) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(H), w2, [0.0]]).astype(np.float32)


def train(X, yc, H=H_DEFAULT, steps=3000, lr=3e-3, seed=0, log=None):
    """Full-batch Adam on the GPU; returns float32 parameters."""
    import torch
    D = X.shape[1]
    dev = torch.device("cuda")
    P = torch.from_numpy(init_params(D, H, seed)).to(dev)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    Xt = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    tt = torch.from_numpy(np.ascontiguousarray(yc, dtype=np.float32)).to(dev)
    losses = []
    for step in range(1, steps + 1):
        loss, g = gz.mlp_loss_grad(P, Xt, tt, H)
        gz.mlp_adam(P, g, m, v, D, H, lr, step)
        losses.append(loss)
        if log and (step % 500 == 0 or step == 1):
            log(f"step {step}: loss {loss:.4f}", flush=True)
    return P.cpu().numpy(), losses


def cv_margin(X, y, grp, folds=5, seed=0, log=None, **kw):
    """The model's validation error in log10 time: groups (one pattern on one
    graph) are dealt to `folds` folds; a network trained on the other folds
    predicts each held-out group, and the root mean square of its centred
    prediction error over all held-out schedules is returned."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    groups = np.unique(grp)
    fold_of = dict(zip(groups, rng.permutation(len(groups)) % folds))
    fold = np.array([fold_of[g] for g in grp])
    yc = centred(y, grp)
    err = np.zeros(len(y))
    for f in range(folds):
        tr, te = fold != f, fold == f
        P, _ = train(X[tr], centred(y[tr], grp[tr]), **kw)
        pred = gz.mlp_forward(torch.from_numpy(P).cuda(),
                              torch.from_numpy(np.ascontiguousarray(X[te], np.float32)).cuda(),
                              kw.get("H", H_DEFAULT), bf16=True).cpu().numpy().astype(np.float64)
        for g in np.unique(grp[te]):
            m = grp[te] == g
            err[np.nonzero(te)[0][m]] = (pred[m] - pred[m].mean()) - yc[te][m]
        if log:
            log(f"fold {f}: held-out rms {np.sqrt(np.mean(err[te] ** 2)):.4f}", flush=True)
    return float(np.sqrt(np.mean(err ** 2)))


def corpus_k_max(X):
    """Largest pattern size among corpus rows: 1 + the loops present (the
    first of each loop's 14 features is its presence flag)."""
    present = np.asarray(X)[:, [14 * i for i in range(7)]] > 0.5
    return int(1 + present.sum(axis=1).max())


# a learned choice must beat the analytic pick's predicted time by this many
# validation errors (two: about 95% confidence for a normal error)
MARGIN_SIGMAS = 2.0


def corpus_graph_range(X):
    """(min, max) of the graph statistics (the last GRAPH_STATS features)
    over the corpus rows."""
    st = np.asarray(X, dtype=np.float32)[:, -gz.GRAPH_STATS:]
    return st.min(axis=0), st.max(axis=0)


def save(params, H, path=MODEL_PATH, margin=0.0, k_max=8, graph_range=None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    extra = {}
    if graph_range is not None:
        extra = dict(graph_min=np.asarray(graph_range[0], np.float32),
                     graph_max=np.asarray(graph_range[1], np.float32))
    np.savez(path, params=np.asarray(params, dtype=np.float32), H=np.int32(H),
             D=np.int32(gz.FEATURES), margin=np.float32(margin), k_max=np.int32(k_max), **extra)


def load(path=MODEL_PATH):
    """(params, H, validation error, k_max, graph range or None); 0, 8 and
    None for a file written without them."""
    z = np.load(path)
    margin = float(z["margin"]) if "margin" in z.files else 0.0
    k_max = int(z["k_max"]) if "k_max" in z.files else 8
    rng = (z["graph_min"], z["graph_max"]) if "graph_min" in z.files else None
    return z["params"].astype(np.float32), int(z["H"]), margin, k_max, rng


def install(path=MODEL_PATH):
    """Install the bundled (or given) model for GZ_SCHED_LEARNED."""
    params, H, err, k_max, rng = load(path)
    gz.set_cost_model(params, H, MARGIN_SIGMAS * err, k_max, rng)
    return params, H


def main(argv):
    if len(argv) >= 2 and argv[0] == "collect":
        collect(argv[1])
    elif len(argv) >= 2 and argv[0] == "train":
        z = np.load(argv[1])
        X, y, grp = z["X"], z["y"], z["group"]
        P, losses = train(X, centred(y, grp), log=print)
        margin = cv_margin(X, y, grp, log=print)
        out = argv[2] if len(argv) > 2 else MODEL_PATH
        save(P, H_DEFAULT, out, margin, corpus_k_max(X), corpus_graph_range(X))
        print(f"saved {out}; final loss {losses[-1]:.4f}, validation error {margin:.4f}")
    elif len(argv) >= 2 and argv[0] == "margin":
        # the validation error of a saved model's training recipe, stored
        # beside its unchanged weights
        z = np.load(argv[1])
        X, y, grp = z["X"], z["y"], z["group"]
        out = argv[2] if len(argv) > 2 else MODEL_PATH
        params, H, _, _, _ = load(out)
        margin = cv_margin(X, y, grp, log=print)
        save(params, H, out, margin, corpus_k_max(X), corpus_graph_range(X))
        print(f"saved {out}; validation error {margin:.4f}, k_max {corpus_k_max(X)}")
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
