"""Connected-pattern enumeration (product side, by vertex augmentation with
numpy canonical codes) and compile-time scaling to all 7-vertex patterns,
on the CPU.

Pins: the oracle's brute-force enumeration (every edge subset, canonical
codes by Python loops) for k <= 5, including the order; the pattern counts
the paper states (112 of 6 vertices, 853 of 7: Section 1); the oracle's
canonical code on sampled 6/7-vertex patterns; and, on sampled 7-vertex
patterns, the library's distinct-schedule count and analytic pick against
the oracle's Algorithm 3 and cost model."""

import json
import os
import sys
import time

import numpy as np
import pytest

from oracle import patterns as P
from paper_1911_12877_amd import gz, motifs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "paper_examples.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)["motif_pattern_counts"]


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_enumeration_matches_oracle_brute_force(k):
    got = motifs.connected_patterns(k)
    want = P.connected_patterns(k)
    # same classes in the same order; representatives may be relabelled
    assert [P.canonical_code(a.tolist()) for a in got] == [P.canonical_code(b) for b in want]


def test_pattern_counts_from_the_paper(golden):
    assert len(motifs.connected_patterns(6)) == golden["6"]
    assert len(motifs.connected_patterns(7)) == golden["7"]
    assert len(motifs.connected_patterns(3)) == golden["3"]
    assert len(motifs.connected_patterns(5)) == golden["5"]


def test_enumerated_patterns_are_connected_and_distinct():
    for k in (6, 7):
        ps = motifs.connected_patterns(k)
        codes = set()
        for a in ps:
            assert P.is_connected(a.tolist())
            codes.add(motifs.canonical_code(a))
        assert len(codes) == len(ps)


def test_canonical_code_matches_oracle():
    rng = np.random.Generator(np.random.PCG64(11))
    for k in (6, 7):
        ps = motifs.connected_patterns(k)
        for i in rng.choice(len(ps), 8, replace=False):
            a = ps[i]
            perm = rng.permutation(k)
            b = a[np.ix_(perm, perm)]  # a relabelled copy
            assert motifs.canonical_code(b) == P.canonical_code(a.tolist())


def test_compile_all_seven_vertex_patterns():
    """Every 7-vertex pattern compiles (automorphisms, Algorithm 3, Algorithm 1
    with Theorem 2, analytic pick); sampled ones agree with the oracle."""
    gz.library()
    ps = motifs.connected_patterns(7)
    t0 = time.perf_counter()
    infos = [gz.compile_pattern(a, True).info() for a in ps]
    dt = time.perf_counter() - t0
    total = sum(i["n_distinct"] for i in infos)
    print(f"compiled {len(ps)} 7-vertex patterns ({total} distinct schedules) "
          f"in {dt:.3f} s", file=sys.stderr)
    rng = np.random.Generator(np.random.PCG64(12))
    for i in rng.choice(len(ps), 6, replace=False):
        a = ps[i].tolist()
        assert infos[i]["n_distinct"] == len(P.distinct_schedules(a))
        order, _ = P.pick_schedule(a, True)
        assert tuple(infos[i]["order"]) == tuple(order)


def test_enumeration_rejects_sizes_out_of_range():
    for k in (1, 8):
        with pytest.raises(ValueError):
            motifs.connected_patterns(k)


def test_oracle_census_identity_seven_vertices():
    """Summed over all 853 connected 7-vertex patterns, the oracle's induced
    counts equal the number of 7-subsets whose induced subgraph is connected
    (brute force over subsets)."""
    import itertools
    import oracle
    from oracle import brute
    from paper_1911_12877_amd import synth
    ps = motifs.connected_patterns(7)
    e = synth.er_edges(12, 0.5, 81)
    O = oracle.from_edge_tuple(e)
    A = brute.dense_adjacency(*e)
    total = sum(oracle.count(O, a.tolist(), True) for a in ps)
    want = sum(P.is_connected(A[np.ix_(s, s)].astype(int).tolist())
               for s in itertools.combinations(range(A.shape[0]), 7))
    assert total == want


def test_named_patterns_match_the_oracles():
    """The product's named patterns are the same graphs (up to labelling)
    as the oracle's, for every name the workloads use."""
    names = ["triangle", "k4", "k5", "c4", "diamond", "tailed_triangle", "house", "k5e",
             "c5", "k6e", "k7e", "c6chord03", "c6chord02", "p4", "star4", "k8", "c8"]
    for nm in names:
        a = motifs.named(nm)
        b = P.named(nm)
        assert motifs.canonical_code(a) == P.canonical_code(b), nm
        # same labelling too, so schedules printed by either side agree
        assert np.array_equal(a, np.array(b, np.uint8)), nm
