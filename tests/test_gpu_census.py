"""GPU checks of the motif census: one captured launch over many graphs and
patterns gives, for every (graph, pattern) pair, the count of a separate
gz_count and of the oracle; replays of the captured graph agree with eager
counts when eager work runs between them; autotuning keeps every count."""

import itertools
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle import patterns as P
from paper_1911_12877_amd import gz, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gz.library()
    yield


def _graphs():
    return [
        ("er12", synth.er_edges(12, 0.4, 901)),
        ("rmat8", synth.rmat_edges(8, 6, seed=902)),
        ("cl400", synth.chung_lu_edges(400, 2.3, 6.0, 903, cap=True)),
        ("er200", synth.er_edges(200, 0.04, 904)),
        ("star30", synth.star_edges(30)),
        ("empty", (np.zeros(0, np.int32), np.zeros(0, np.int32), 9)),
    ]


def _patterns():
    pats = [P.named("p2")]
    for k in (3, 4, 5):
        pats += P.connected_patterns(k)
    return pats


@pytest.fixture(scope="module")
def census_case():
    gl = _graphs()
    G = [gz.load_edges(*e) for _, e in gl]
    pats = _patterns()
    S = [gz.compile_pattern(a, True) for a in pats]
    return gl, G, pats, S


def test_census_matches_counts_and_oracle(census_case):
    gl, G, pats, S = census_case
    c = gz.Census(G, S)
    counts, ms = c.run()
    print(f"census {len(G)} graphs x {len(S)} patterns in {ms:.2f} ms", file=sys.stderr)
    for gi, (name, e) in enumerate(gl):
        O = oracle.from_edge_tuple(e)
        for si, a in enumerate(pats):
            want = oracle.count(O, a, True)
            assert int(counts[gi, si]) == want, (name, a)
            assert gz.count(G[gi], S[si]) == want


def test_census_graph_replays_with_eager_work_between(census_case):
    gl, G, pats, S = census_case
    c = gz.Census(G, S)
    eager = np.array([[gz.count(g, s) for s in S] for g in G], dtype=np.uint64)
    for rep in range(3):
        got, _ = c.run()
        assert np.array_equal(got, eager), rep
        # eager work of the program between replays
        assert gz.count(G[1], S[-1]) == int(eager[1, -1])
        import torch
        torch.cuda.synchronize()


def test_census_tune_keeps_counts(census_case):
    gl, G, pats, S = census_case
    c = gz.Census(G, S)
    before, _ = c.run()
    params, best = c.tune()
    assert params[0] in (8, 32, 128) and params[1] in (1, 4, 16) and params[2] in (1, 4)
    after, _ = c.run()
    assert np.array_equal(before, after)


def test_census_connected_subsets_identity():
    """Summed over all connected k-vertex patterns, induced counts equal the
    number of k-subsets whose induced subgraph is connected (brute force)."""
    e = synth.er_edges(13, 0.35, 905)
    A = brute.dense_adjacency(*e)
    G = gz.load_edges(*e)
    for k in (3, 4, 5):
        pats = P.connected_patterns(k)
        S = [gz.compile_pattern(a, True) for a in pats]
        counts, _ = gz.Census([G], S).run()
        want = 0
        for sub in itertools.combinations(range(A.shape[0]), k):
            sub_adj = A[np.ix_(sub, sub)].astype(int).tolist()
            want += P.is_connected(sub_adj)
        assert int(counts.sum()) == want, k


def test_census_mixes_size_classes():
    """Patterns of 3-5 and of 6 vertices in one census: both kernels of the
    captured graph run and each pair keeps its own count."""
    e = synth.er_edges(13, 0.4, 906)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    pats = [P.named("c6"), P.named("triangle"), P.named("k6e"), P.named("house")]
    counts, _ = gz.Census([G], [gz.compile_pattern(a, True) for a in pats]).run()
    for i, a in enumerate(pats):
        assert int(counts[0, i]) == oracle.count(O, a, True), i
