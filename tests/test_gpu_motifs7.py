"""GPU parity for every connected 6- and 7-vertex pattern: single counts
against the oracle, and the census over 6/7-vertex patterns (its second size
class) against single counts, replays, and the connected-subset identity
(brute force over vertex subsets)."""

import itertools
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle import patterns as P
from paper_1911_12877_amd import gz, motifs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gz.library()
    yield


def _connected_subsets(e, k):
    A = brute.dense_adjacency(*e)
    return sum(P.is_connected(A[np.ix_(s, s)].astype(int).tolist())
               for s in itertools.combinations(range(A.shape[0]), k))


def test_all_seven_vertex_patterns_against_oracle():
    ps = motifs.connected_patterns(7)
    e = synth.er_edges(12, 0.5, 81)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    total = 0
    for i, a in enumerate(ps):
        got = gz.count(G, gz.compile_pattern(a, True))
        assert got == oracle.count(O, a.tolist(), True), i
        total += got
    assert total == _connected_subsets(e, 7)


def test_census_six_and_seven_vertex_patterns():
    graphs = [synth.er_edges(12, 0.5, 81), synth.er_edges(13, 0.35, 82),
              synth.chung_lu_edges(60, 2.3, 8.0, 83, cap=False)]
    G = [gz.load_edges(*e) for e in graphs]
    pats = motifs.connected_patterns(6) + motifs.connected_patterns(7) + \
        motifs.connected_patterns(4)
    S = [gz.compile_pattern(a, True) for a in pats]
    c = gz.Census(G, S)
    counts, ms = c.run()
    print(f"census {len(G)} graphs x {len(S)} patterns (4, 6 and 7 vertices) in "
          f"{ms:.2f} ms", file=sys.stderr, flush=True)
    for gi, g in enumerate(G):
        for si, s in enumerate(S):
            assert int(counts[gi, si]) == gz.count(g, s), (gi, si)
    n6, n7 = 112, 853
    for gi, e in enumerate(graphs[:2]):
        assert int(counts[gi, :n6].sum()) == _connected_subsets(e, 6)
        assert int(counts[gi, n6:n6 + n7].sum()) == _connected_subsets(e, 7)
    again, _ = c.run()
    assert np.array_equal(again, counts)


def test_census_rejects_eight_vertex_patterns():
    G = gz.load_edges(*synth.cycle_edges(10))
    with pytest.raises(gz.GzError) as ex:
        gz.Census([G], [gz.compile_pattern(P.named("c8"), True)])
    assert ex.value.status == gz.GZ_ENOTSUP
