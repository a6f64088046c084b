"""Seeded synthetic input graphs.

This module is the one piece shared by the product path and the oracle: it only
draws edge lists.  It holds none of the mining method's arithmetic (no
normalisation, reindexing, pattern handling or counting); every consumer turns
the raw edge list into a simple graph with its own code.

The paper evaluates on real graphs (its Table 1) that are not available here;
the generators below stand in for them with the shapes the evaluation needs:
a small uniform graph, power-law R-MAT graphs and Chung-Lu graphs.

All generators return ``(src, dst, n)`` with int32 endpoint arrays.  The lists
are raw: they may contain self-loops, duplicates and both orientations of an
edge.  Randomness comes from numpy's PCG64 bit generator seeded with the given
integer, so a (generator, parameters, seed) triple names one edge list.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "er_edges", "rmat_edges", "chung_lu_edges", "chung_lu_weights",
    "complete_edges", "complete_bipartite_edges", "cycle_edges", "path_edges",
    "star_edges", "petersen_edges", "hypercube_edges", "grid_edges",
    "config_graph", "CONFIGS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def er_edges(n: int, p: float, seed: int):
    """Erdos-Renyi G(n, p): each unordered pair {i, j}, i < j, is an edge with
    probability p, decided by one uniform double per pair in row-major (i, j)
    order."""
    rng = _rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.shape[0]) < p
    return iu[keep].astype(np.int32), ju[keep].astype(np.int32), int(n)


def rmat_edges(scale: int, edge_factor: int = 16,
               abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 0,
               chunk: int = 1 << 23):
    """R-MAT sampler: ``edge_factor * 2**scale`` samples on ``n = 2**scale``
    vertices.  For every sample and every one of the ``scale`` bit levels a
    32-bit uniform integer picks a quadrant with probabilities (a, b, c, d):
    a -> (0,0), b -> (0,1), c -> (1,0), d -> (1,1) for (src bit, dst bit),
    most significant bit first.  No noise and no vertex permutation.
    Thresholds are the cumulative probabilities rounded to 32-bit integers."""
    a, b, c, d = abcd
    n = 1 << scale
    m = edge_factor * n
    t1 = np.uint32(min(round(a * 2**32), 2**32 - 1))
    t2 = np.uint32(min(round((a + b) * 2**32), 2**32 - 1))
    t3 = np.uint32(min(round((a + b + c) * 2**32), 2**32 - 1))
    rng = _rng(seed)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.int32)
        t = np.zeros(hi - lo, dtype=np.int32)
        for level in range(scale):
            r = rng.integers(0, 2**32, size=hi - lo, dtype=np.uint32)
            sbit = r >= t2                      # quadrants c, d
            dbit = ((r >= t1) & (r < t2)) | (r >= t3)  # quadrants b, d
            shift = scale - 1 - level
            s |= sbit.astype(np.int32) << shift
            t |= dbit.astype(np.int32) << shift
        src[lo:hi] = s
        dst[lo:hi] = t
    return src, dst, int(n)


def chung_lu_weights(n: int, gamma: float, avg_deg: float, cap: bool = True):
    """Expected-degree weights w_i proportional to (i+1)^(-1/(gamma-1)),
    scaled to mean ``avg_deg``; with ``cap`` every weight is clipped at
    sqrt(sum w) so that w_i w_j / sum(w) <= 1 (the Chung-Lu admissibility
    condition)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    w = i ** (-1.0 / (gamma - 1.0))
    w *= avg_deg * n / w.sum()
    if cap:
        w = np.minimum(w, np.sqrt(w.sum()))
    return w


def chung_lu_edges(n: int, gamma: float, avg_deg: float, seed: int,
                   cap: bool = True):
    """Chung-Lu power-law graph: ``m = round(n * avg_deg / 2)`` samples, each
    endpoint drawn independently with probability proportional to its weight
    (inverse-CDF on one uniform double per endpoint)."""
    w = chung_lu_weights(n, gamma, avg_deg, cap)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(n * avg_deg / 2.0))
    rng = _rng(seed)
    u = rng.random(2 * m)
    ends = np.searchsorted(cdf, u, side="right")
    ends = np.minimum(ends, n - 1).astype(np.int32)
    return ends[:m].copy(), ends[m:].copy(), int(n)


# ---------------------------------------------------------------- structured

def _pairs(pairs, n):
    if len(pairs) == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32), int(n)
    a = np.asarray(pairs, dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy(), int(n)


def complete_edges(n: int):
    return _pairs([(i, j) for i in range(n) for j in range(i + 1, n)], n)


def complete_bipartite_edges(a: int, b: int):
    return _pairs([(i, a + j) for i in range(a) for j in range(b)], a + b)


def cycle_edges(n: int):
    return _pairs([(i, (i + 1) % n) for i in range(n)], n)


def path_edges(n: int):
    return _pairs([(i, i + 1) for i in range(n - 1)], n)


def star_edges(leaves: int):
    """Vertex 0 is the hub, 1..leaves are leaves."""
    return _pairs([(0, i) for i in range(1, leaves + 1)], leaves + 1)


def petersen_edges():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return _pairs(outer + spokes + inner, 10)


def hypercube_edges(d: int):
    n = 1 << d
    return _pairs([(v, v ^ (1 << b)) for v in range(n) for b in range(d)
                   if v < v ^ (1 << b)], n)


def grid_edges(r: int, c: int):
    pairs = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                pairs.append((v, v + 1))
            if i + 1 < r:
                pairs.append((v, v + c))
    return _pairs(pairs, r * c)


# ---------------------------------------------------------- named workloads

CONFIGS = {
    # small uniform graph: triangles (exact, checked in full by the oracle)
    "er2000": dict(kind="er", n=2000, p=0.008, seed=1001),
    # power-law graph for k-clique counts
    "rmat20": dict(kind="rmat", scale=20, edge_factor=16, seed=2001),
    # larger power-law graph for the vertex-induced non-clique patterns
    "rmat22": dict(kind="rmat", scale=22, edge_factor=16, seed=3001),
    # learned-schedule graphs
    "rmat21": dict(kind="rmat", scale=21, edge_factor=16, seed=5001),
    "cl2m": dict(kind="chung_lu", n=2_000_000, gamma=2.2, avg_deg=16.0,
                 seed=5002),
}


def census_graph_params(index: int):
    """Parameters of graph ``index`` (0..63) of the motif-census batch:
    exponent U[2.1, 2.8], n log-uniform in [1e3, 2e5], average degree
    U[8, 32], drawn from a PCG64 stream seeded with 40000+index; the edge list
    itself uses seed 4001+index."""
    rng = _rng(40000 + index)
    gamma = float(rng.uniform(2.1, 2.8))
    n = int(10 ** rng.uniform(3.0, np.log10(2e5)))
    avg_deg = float(rng.uniform(8.0, 32.0))
    return dict(kind="chung_lu", n=n, gamma=gamma, avg_deg=avg_deg,
                seed=4001 + index)


def config_graph(name_or_params):
    """Edge list of a named workload (see ``CONFIGS``) or of a parameter dict."""
    p = CONFIGS[name_or_params] if isinstance(name_or_params, str) else name_or_params
    kind = p["kind"]
    if kind == "er":
        return er_edges(p["n"], p["p"], p["seed"])
    if kind == "rmat":
        return rmat_edges(p["scale"], p.get("edge_factor", 16),
                          p.get("abcd", (0.57, 0.19, 0.19, 0.05)), p["seed"])
    if kind == "chung_lu":
        return chung_lu_edges(p["n"], p["gamma"], p["avg_deg"], p["seed"],
                              p.get("cap", True))
    raise ValueError(f"unknown graph kind {kind!r}")
