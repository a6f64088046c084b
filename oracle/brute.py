"""Oracle tier 0: brute force, straight from the definition of the count.
TEST INFRASTRUCTURE ONLY.

For a simple graph G and a pattern P on k vertices:
* vertex-induced count = number of k-subsets S of V with G[S] isomorphic to P;
* edge-induced count   = number of subgraphs H of G isomorphic to P
                       = (number of (S, bijection) pairs that map every
                          pattern edge onto a graph edge) / |Aut(P)|.

Every k-subset is enumerated; its induced subgraph is encoded as a bit string
over the k(k-1)/2 position pairs and matched against the codes of all k!
placements of P.  Feasible for n up to a few dozen.  Shares no code with the
rest of the oracle.
"""

from __future__ import annotations

import itertools

import numpy as np


def dense_adjacency(src, dst, n):
    """Boolean adjacency of the simple graph behind a raw edge list."""
    A = np.zeros((n, n), dtype=bool)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    A[src, dst] = True
    A[dst, src] = True
    np.fill_diagonal(A, False)
    return A


def _pair_index(k):
    return [(a, b) for a in range(k) for b in range(a + 1, k)]


def _placement_codes(P):
    """Code of every placement of P on positions 0..k-1 (one per bijection)."""
    k = len(P)
    pairs = _pair_index(k)
    bit = {pr: i for i, pr in enumerate(pairs)}
    codes = []
    for pi in itertools.permutations(range(k)):
        c = 0
        for p in range(k):
            for q in range(p + 1, k):
                if P[p][q]:
                    a, b = sorted((pi[p], pi[q]))
                    c |= 1 << bit[(a, b)]
        codes.append(c)
    return codes


def aut_size(P):
    codes = _placement_codes(P)
    return sum(1 for c in codes if c == codes[0])


def _subset_codes(A, k, chunk=200_000):
    n = A.shape[0]
    pairs = _pair_index(k)
    it = itertools.combinations(range(n), k)
    while True:
        block = list(itertools.islice(it, chunk))
        if not block:
            return
        S = np.array(block, dtype=np.int64)
        code = np.zeros(S.shape[0], dtype=np.int64)
        for i, (a, b) in enumerate(pairs):
            code |= A[S[:, a], S[:, b]].astype(np.int64) << i
        yield code


def count(A, P, induced=True):
    """Exact count by enumeration of all k-subsets (A: dense boolean
    adjacency, P: k x k 0/1 pattern)."""
    k = len(P)
    if k > A.shape[0]:
        return 0
    codes = _placement_codes(P)
    npairs = k * (k - 1) // 2
    if induced:
        table = np.zeros(1 << npairs, dtype=np.int64)
        for c in set(codes):
            table[c] = 1
        return int(sum(int(table[c].sum()) for c in _subset_codes(A, k)))
    # edge-induced: placements whose edges are all present, over |Aut|
    allc = np.arange(1 << npairs, dtype=np.int64)
    table = np.zeros(1 << npairs, dtype=np.int64)
    for c in set(codes):
        table += codes.count(c) * ((allc & c) == c).astype(np.int64)
    total = sum(int(table[c].sum()) for c in _subset_codes(A, k))
    aut = aut_size(P)
    assert total % aut == 0
    return total // aut
