"""Connected patterns (motifs) of k vertices up to isomorphism, for the
census and for compile-time scaling.

Every connected graph on k vertices has a vertex whose removal leaves it
connected (a leaf of a spanning tree), so the connected k-vertex graphs are
the connected (k-1)-vertex graphs plus one vertex joined to a non-empty
subset of them.  Each candidate is reduced to its canonical code, the
largest upper-triangle bit string over all k! relabellings (evaluated for all
relabellings at once with numpy), and duplicates are dropped.  Patterns are
returned in (edge count, canonical code) order, the order the census uses.
"""

from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def _tables(k):
    perms = np.array(list(itertools.permutations(range(k))), dtype=np.int64)
    ii, jj = np.triu_indices(k, 1)
    weights = (np.int64(1) << np.arange(len(ii) - 1, -1, -1, dtype=np.int64))
    return perms[:, ii], perms[:, jj], weights


def canonical_code(adj) -> int:
    """Largest upper-triangle bit string (row-major, first pair most
    significant) of adj over all relabellings."""
    a = np.asarray(adj, dtype=np.int64)
    pi, pj, w = _tables(a.shape[0])
    return int((a[pi, pj] @ w).max())


def from_code(k, code):
    """The adjacency matrix whose upper-triangle bit string is `code`."""
    ii, jj = np.triu_indices(k, 1)
    a = np.zeros((k, k), dtype=np.uint8)
    n = len(ii)
    for b in range(n):
        if (code >> (n - 1 - b)) & 1:
            a[ii[b], jj[b]] = a[jj[b], ii[b]] = 1
    return a


@lru_cache(maxsize=None)
def _codes(k):
    if k < 2:
        raise ValueError("patterns need at least 2 vertices")
    if k == 2:
        return (1,)
    seen = set()
    for c in _codes(k - 1):
        base = from_code(k - 1, c)
        for mask in range(1, 1 << (k - 1)):
            a = np.zeros((k, k), dtype=np.uint8)
            a[:k - 1, :k - 1] = base
            for v in range(k - 1):
                if (mask >> v) & 1:
                    a[v, k - 1] = a[k - 1, v] = 1
            seen.add(canonical_code(a))
    return tuple(sorted(seen, key=lambda c: (bin(c).count("1"), c)))


def connected_patterns(k):
    """All connected k-vertex patterns up to isomorphism (2 <= k <= 7), as
    uint8 adjacency matrices, in (edge count, canonical code) order; k = 7
    (853 patterns) takes a few seconds."""
    if not 2 <= k <= 7:
        raise ValueError("pattern size must be between 2 and 7")
    return [from_code(k, c) for c in _codes(k)]


def _adj(k, edges):
    a = np.zeros((k, k), dtype=np.uint8)
    for u, v in edges:
        a[u, v] = a[v, u] = 1
    return a


def named(name):
    """Adjacency (uint8) of a named pattern: 'triangle', 'diamond' (K4 minus
    the edge {2,3}), 'tailed_triangle' (triangle 0-1-2 with 3 joined to 0),
    'house' (4-cycle 0-1-2-3 with 4 joined to 0 and 1), 'k<n>', 'k<n>e' (K_n
    minus the edge {n-2, n-1}), 'c<n>' (cycle), 'p<n>' (path), 'star<n>' (hub
    0 and n-1 leaves), 'c6chord03' / 'c6chord02' (6-cycle with the chord
    {0,3} / {0,2})."""
    ring = lambda n: [(i, (i + 1) % n) for i in range(n)]
    fixed = {
        "triangle": (3, [(0, 1), (1, 2), (0, 2)]),
        "diamond": (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)]),
        "tailed_triangle": (4, [(0, 1), (1, 2), (0, 2), (0, 3)]),
        "house": (5, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4)]),
        "c6chord03": (6, ring(6) + [(0, 3)]),
        "c6chord02": (6, ring(6) + [(0, 2)]),
    }
    if name in fixed:
        return _adj(*fixed[name])
    for prefix, make in (("star", lambda n: [(0, i) for i in range(1, n)]),
                         ("k", lambda n: [(i, j) for i in range(n) for j in range(i + 1, n)]),
                         ("c", ring),
                         ("p", lambda n: [(i, i + 1) for i in range(n - 1)])):
        rest = name[len(prefix):]
        if name.startswith(prefix) and rest.isdigit():
            return _adj(int(rest), make(int(rest)))
    if name.startswith("k") and name.endswith("e") and name[1:-1].isdigit():
        n = int(name[1:-1])
        return _adj(n, [(i, j) for i in range(n) for j in range(i + 1, n)
                        if (i, j) != (n - 2, n - 1)])
    raise KeyError(name)
