"""GPU parity: libgz's HIP mining path against the oracle, bit-exact, on
seeded inputs small enough for the oracle to count in full (several tiles,
ragged tails, hubs longer than one materialised chunk), plus the invariants
the method must keep whatever schedule, bound set or labelling it runs."""

import math
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


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(e, reindex=True):
    flags = 0 if reindex else gz.GRAPH_NO_REINDEX
    return gz.load_edges(*e, flags=flags), oracle.from_edge_tuple(e, reindex)


def _tiny_graphs():
    yield "er14", synth.er_edges(14, 0.45, 1)
    yield "er16", synth.er_edges(16, 0.30, 2)
    yield "rmat4", synth.rmat_edges(4, 6, seed=3)
    yield "cl18", synth.chung_lu_edges(18, 2.3, 6.0, 4, cap=False)
    yield "k9", synth.complete_edges(9)
    yield "petersen", synth.petersen_edges()
    yield "star12", synth.star_edges(12)
    yield "c11", synth.cycle_edges(11)


@pytest.mark.parametrize("k", [2, 3, 4, 5])
@pytest.mark.parametrize("induced", [True, False])
def test_tiny_graphs_all_patterns(k, induced):
    for name, e in _tiny_graphs():
        _say("tiny", name, k, induced)
        G, O = _pair(e)
        for pat in P.connected_patterns(k):
            want = oracle.count(O, pat, induced)
            got = gz.count(G, gz.compile_pattern(pat, induced))
            assert got == want, (name, pat, induced)


@pytest.mark.parametrize("name", ["k6", "k6e", "c6", "c6chord03", "c6chord02", "k7e", "c7",
                                  "k7", "star6", "p6"])
def test_larger_patterns_small_dense(name):
    pat = P.named(name)
    for seed, p in ((5, 0.55), (6, 0.75)):
        e = synth.er_edges(13, p, seed)
        _say("larger", name, seed)
        G, O = _pair(e)
        for induced in (True, False):
            assert gz.count(G, gz.compile_pattern(pat, induced)) == oracle.count(O, pat, induced)


def test_eight_vertex_patterns():
    for nm, pat in (("c8", P.named("c8")), ("k8e", P.named("k8e")), ("p8", P.named("p8"))):
        e = synth.er_edges(12, 0.7, 9)
        _say("k8", nm)
        G, O = _pair(e)
        for induced in (True, False):
            assert gz.count(G, gz.compile_pattern(pat, induced)) == oracle.count(O, pat, induced)


MEDIUM = ["triangle", "k4", "k5", "c4", "diamond", "tailed_triangle", "house", "k5e", "c5",
          "p4", "star4"]


def _medium_graphs():
    # hubs of the R-MAT graph exceed one materialised chunk (256 elements)
    yield "rmat10", synth.rmat_edges(10, 8, seed=21)
    yield "cl2000", synth.chung_lu_edges(2000, 2.3, 8.0, 22, cap=True)
    yield "er400", synth.er_edges(400, 0.03, 23)


@pytest.mark.parametrize("gname", ["rmat10", "cl2000", "er400"])
def test_medium_graphs(gname):
    e = dict(_medium_graphs())[gname]
    G, O = _pair(e)
    for nm in MEDIUM:
        for induced in (True, False):
            _say("medium", gname, nm, induced)
            pat = P.named(nm)
            assert gz.count(G, gz.compile_pattern(pat, induced)) == \
                oracle.count(O, pat, induced), (gname, nm, induced)


def test_exported_graph_is_oracle_reindex():
    e = synth.rmat_edges(12, 16, seed=31)
    G, O = _pair(e)
    r, c, old_of_new = gz.graph_export(G)
    assert np.array_equal(r, O.rowptr.astype(np.int32))
    assert np.array_equal(c, O.col)
    assert np.array_equal(O.new_of_old[old_of_new], np.arange(O.n))


@pytest.mark.parametrize("nm", ["k4", "c4", "tailed_triangle", "house", "k5e", "diamond"])
def test_per_root_parity(nm):
    e = synth.chung_lu_edges(3000, 2.2, 12.0, 41, cap=False)
    G, O = _pair(e)
    pat = P.named(nm)
    s = gz.compile_pattern(pat, True)
    info = s.info()
    roots = np.arange(O.n, dtype=np.int32)
    got = gz.count_roots(G, s, roots)
    total, want = oracle.count(O, pat, True, order=info["order"], relations="thm2",
                               roots=roots, per_root=True)
    assert np.array_equal(got, want)
    assert int(got.sum()) == total == gz.count(G, s)
    # a shuffled subset with repeats
    rng = np.random.Generator(np.random.PCG64(7))
    sub = rng.integers(0, O.n, 500).astype(np.int32)
    assert np.array_equal(gz.count_roots(G, s, sub), want[sub])


@pytest.mark.parametrize("nm", ["house", "c5", "diamond", "k5e", "tailed_triangle"])
def test_schedule_invariance_and_theorem1(nm):
    pat = P.named(nm)
    e = synth.chung_lu_edges(1500, 2.3, 10.0, 51, cap=True)
    G, O = _pair(e)
    aut = P.multiplicity(pat)
    for induced in (True, False):
        want = oracle.count(O, pat, induced)
        for order, _ in gz.enumerate_schedules(pat, induced):
            assert gz.count(G, gz.compile_pattern_order(pat, order, induced)) == want
        nr = gz.compile_pattern(pat, induced, gz.SCHED_NO_RESTRICT)
        assert gz.count(G, nr) == aut * want


def test_orientation_off_same_counts():
    e = synth.rmat_edges(11, 16, seed=61)
    G1 = gz.load_edges(*e)
    G2 = gz.load_edges(*e, flags=gz.GRAPH_NO_REINDEX)
    for nm in ["k4", "c4", "house", "tailed_triangle"]:
        s = gz.compile_pattern(P.named(nm), True)
        assert gz.count(G1, s) == gz.count(G2, s)


@pytest.mark.parametrize("nm", ["triangle", "k4", "c4", "house", "k5e", "tailed_triangle"])
def test_instrumented_bytes(nm):
    e = synth.chung_lu_edges(2000, 2.3, 10.0, 71, cap=True)
    G, O = _pair(e)
    pat = P.named(nm)
    for induced in (True, False):
        s = gz.compile_pattern(pat, induced)
        info = s.info()
        b, c = gz.count_bytes(G, s)
        ob, oc = oracle.instrument(O, pat, induced, info["order"], info["bound"])
        assert (b, c) == (ob, oc)


def test_edge_cases():
    tri = gz.compile_pattern(P.named("triangle"), True)
    edge = gz.compile_pattern(P.named("p2"), True)
    # no edges at all
    G = gz.load_edges(np.zeros(0, np.int32), np.zeros(0, np.int32), 5)
    assert gz.count(G, tri) == 0 and gz.count(G, edge) == 0
    # only self-loops and duplicates of one edge
    G = gz.load_edges(np.array([0, 1, 1, 2], np.int32), np.array([0, 2, 2, 1], np.int32), 3)
    assert gz.count(G, edge) == 1 and gz.count(G, tri) == 0
    # reindexed: old 1 -> 0, old 2 -> 1, old 0 -> 2; the edge {0,1} is found
    # from its larger-id end (the bound makes loop 1 smaller than loop 0)
    assert list(gz.count_roots(G, edge, np.array([0, 1, 2], np.int32))) == [0, 1, 0]
    # one vertex
    G = gz.load_edges(np.zeros(0, np.int32), np.zeros(0, np.int32), 1)
    assert gz.count(G, tri) == 0
    # the edge pattern counts edges
    e = synth.rmat_edges(10, 8, seed=81)
    G, O = _pair(e)
    assert gz.count(G, edge) == O.col.shape[0] // 2
    # complete graphs: closed forms
    for n in (12, 40):
        G = gz.load_edges(*synth.complete_edges(n))
        for k in (3, 4, 5):
            assert gz.count(G, gz.compile_pattern(P.named(f"k{k}"), True)) == math.comb(n, k)
        assert gz.count(G, gz.compile_pattern(P.named("c4"), True)) == 0
        assert gz.count(G, gz.compile_pattern(P.named("c4"), False)) == 3 * math.comb(n, 4)
    # a hub far longer than one chunk, probed from every side
    G = gz.load_edges(*synth.star_edges(2000))
    for k in (3, 4):
        got = gz.count(G, gz.compile_pattern(P.named(f"star{k}"), True))
        assert got == math.comb(2000, k - 1)
    G = gz.load_edges(*synth.complete_bipartite_edges(30, 700))
    assert gz.count(G, gz.compile_pattern(P.named("c4"), True)) == \
        math.comb(30, 2) * math.comb(700, 2)


def test_triangles_uniform_2000():
    e = synth.config_graph("er2000")
    G, O = _pair(e)
    A = brute.dense_adjacency(*e).astype(np.float64)
    want = int(round(np.trace(A @ A @ A) / 6.0))
    assert oracle.count(O, P.named("triangle")) == want
    assert gz.count(G, gz.compile_pattern(P.named("triangle"), True)) == want


def test_device_pointer_inputs_and_stream():
    import torch
    e = synth.chung_lu_edges(5000, 2.4, 10.0, 91, cap=True)
    s = torch.cuda.Stream()
    src = torch.from_numpy(e[0]).cuda()
    dst = torch.from_numpy(e[1]).cuda()
    torch.cuda.synchronize()
    G = gz.load_edges(src, dst, e[2], stream=s)
    O = oracle.from_edge_tuple(e)
    r = torch.from_numpy(O.rowptr.astype(np.int32)).cuda()
    c = torch.from_numpy(O.col).cuda()
    torch.cuda.synchronize()
    G2 = gz.load_graph(r, c, flags=0, stream=s)
    for nm in ["k4", "house"]:
        sc = gz.compile_pattern(P.named(nm), True)
        want = oracle.count(O, P.named(nm), True)
        assert gz.count(G, sc, stream=s) == want
        assert gz.count(G2, sc, stream=s) == want


def test_strict_csr_rejects_malformed():
    r = np.array([0, 1, 1], np.int32)
    c = np.array([1], np.int32)  # 0->1 without 1->0
    with pytest.raises(gz.GzError) as ex:
        gz.load_graph(r, c, flags=0)
    assert ex.value.status == gz.GZ_EINVAL
    G = gz.load_graph(r, c, flags=gz.GRAPH_NORMALIZE)
    assert gz.graph_info(G)["nnz"] == 2


def test_clique_paths_closed_forms():
    """K_n: every C2 has n-2 elements, so n = 120 sends every edge with
    C2 > 64 elements through the workgroup path with two-word rows."""
    for n in (40, 120):
        G = gz.load_edges(*synth.complete_edges(n))
        for k in (5, 6, 7, 8):
            _say("clique closed form", n, k)
            assert gz.count(G, gz.compile_pattern(P.named(f"k{k}"), True)) == math.comb(n, k)


def test_clique_widest_rows_closed_forms():
    """K_700: after reindexing root v has the v candidates 0..v-1, so roots
    above 512 build rows of 9 to 11 words, the widest size class.  Totals
    are C(700, k) and the count of root v is C(v, k - 1): the k-cliques whose
    largest id is v."""
    n = 700
    G = gz.load_edges(*synth.complete_edges(n))
    roots = np.arange(n, dtype=np.int32)
    for k in (4, 5):
        s = gz.compile_pattern(P.named(f"k{k}"), True)
        _say("K_700 clique closed form", k)
        assert gz.count(G, s) == math.comb(n, k)
        per = gz.count_roots(G, s, roots)
        want = np.array([math.comb(v, k - 1) for v in range(n)], dtype=np.uint64)
        assert np.array_equal(per, want), k
    assert math.comb(n, 4) == 9_918_641_075 and math.comb(n, 5) == 1_380_674_837_640


def test_clique_roots_over_capacity_take_generic_loops():
    """Bit rows hold at most 1024 candidates: on K_1040 the roots 1025..1039
    take the generic loops through a root list while the others stay on the
    clique kernels, and per-root counts land in their own slots.  The gate
    is also forced low (GZ_CLIQUE_MAX_LO) so that most roots of K_300 and of
    an R-MAT graph cross it."""
    import os
    n = 1040
    G = gz.load_edges(*synth.complete_edges(n))
    s = gz.compile_pattern(P.named("k4"), True)
    assert gz.count(G, s) == math.comb(n, 4)
    roots = np.array([3, 1039, 500, 1030, 1024, 1025, 7], np.int32)
    want = np.array([math.comb(int(v), 3) for v in roots], dtype=np.uint64)
    assert np.array_equal(gz.count_roots(G, s, roots), want)
    try:
        os.environ["GZ_CLIQUE_MAX_LO"] = "100"
        G = gz.load_edges(*synth.complete_edges(300))
        for k in (4, 5):
            s = gz.compile_pattern(P.named(f"k{k}"), True)
            assert gz.count(G, s) == math.comb(300, k), k
            per = gz.count_roots(G, s, np.arange(300, dtype=np.int32))
            assert np.array_equal(per, np.array([math.comb(v, k - 1) for v in range(300)],
                                                dtype=np.uint64)), k
        e = synth.rmat_edges(10, 16, seed=114)
        G, O = _pair(e)
        roots = np.arange(O.n, dtype=np.int32)
        for gate in ("0", "8", "40"):
            os.environ["GZ_CLIQUE_MAX_LO"] = gate
            for k in (4, 5):
                pat = P.named(f"k{k}")
                s = gz.compile_pattern(pat, True)
                total, per = oracle.count(O, pat, True, order=s.info()["order"], relations="thm2",
                                          roots=roots, per_root=True)
                assert gz.count(G, s) == total, (gate, k)
                assert np.array_equal(gz.count_roots(G, s, roots), per), (gate, k)
    finally:
        os.environ.pop("GZ_CLIQUE_MAX_LO", None)


@pytest.mark.parametrize("which", ["er_dense", "rmat10", "cl_core"])
def test_clique_paths_vs_oracle(which):
    if which == "er_dense":
        e = synth.er_edges(200, 0.5, 111)
    elif which == "rmat10":
        e = synth.rmat_edges(10, 16, seed=112)
    else:
        e = synth.chung_lu_edges(3000, 2.1, 24.0, 113, cap=False)
    G, O = _pair(e)
    _say("clique vs oracle", which, gz.graph_info(G))
    for k in (5, 6, 7):
        pat = P.named(f"k{k}")
        s = gz.compile_pattern(pat, True)
        want = oracle.count(O, pat, True)
        assert gz.count(G, s) == want, (which, k)
        roots = np.arange(O.n, dtype=np.int32)
        _, per = oracle.count(O, pat, True, order=s.info()["order"], relations="thm2",
                              roots=roots, per_root=True)
        assert np.array_equal(gz.count_roots(G, s, roots), per), (which, k)


def _clique_ops_complete(n, k):
    """Lane operations of the bit-row intersections for K_k on K_n, from the
    definition: after reindexing vertex v has lo = v candidates and every row
    is full (row p = bits 0..p-1).  A row-word intersection of r rows costs
    2(r-1); the last level adds 2 for the popcount."""
    import functools

    def words(p):  # words holding bits below p
        return (p + 63) // 64

    @functools.lru_cache(maxsize=None)
    def cl_w(depth, r, b, nw):
        # the AND of r rows including row b (bits < b), over words [0, nw)
        ops = 0
        for w in range(nw):
            ops += 2 * (r - 1) + (2 if depth == 0 else 0)
            if depth > 0:
                for c in range(64 * w, min(64 * w + 64, b)):
                    ops += cl_w(depth - 1, r + 1, c, w + 1)
        return ops

    total = 0
    for d in range(k - 1, n):  # roots with fewer than k-1 candidates are skipped
        for a in range(d):
            for w in range(words(a)):
                for b in range(64 * w, min(64 * w + 64, a)):
                    total += cl_w(k - 4, 2, b, w + 1)
    return total


def test_clique_op_count_definition():
    for n, k in ((30, 4), (30, 5), (90, 4), (70, 5)):
        G = gz.load_edges(*synth.complete_edges(n))
        s = gz.compile_pattern(P.named(f"k{k}"), True)
        ops, c = gz.count_ops(G, s)
        assert c == math.comb(n, k)
        assert ops == _clique_ops_complete(n, k), (n, k)
    G = gz.load_edges(*synth.cycle_edges(10))
    with pytest.raises(gz.GzError) as ex:
        gz.count_ops(G, gz.compile_pattern(P.named("c4"), True))
    assert ex.value.status == gz.GZ_ENOTSUP
