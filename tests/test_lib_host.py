"""Host-side checks of libgz that need no GPU: the library loads and exports
every symbol its header declares, the pattern compiler agrees with the
oracle's restatement of the paper's algorithms, host graph preparation agrees
with the oracle's, and malformed input is rejected with clean errors."""

import os
import re

import numpy as np
import pytest

import oracle
from oracle import patterns as P
from paper_1911_12877_amd import gz, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gz.LIB_PATH):
        from paper_1911_12877_amd import build
        build.build()
    return gz.library()


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "gz.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gz_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert len(syms) >= 15
    for name in syms:
        assert hasattr(lib, name), name


NAMED = ["triangle", "k4", "k5", "c4", "c5", "c6", "diamond", "tailed_triangle", "house",
         "k5e", "k6e", "k7e", "c6chord03", "c6chord02", "p4", "p5", "star4", "star5"]


def _all_patterns():
    for k in (2, 3, 4, 5):
        for a in P.connected_patterns(k):
            yield a
    for nm in NAMED:
        yield P.named(nm)


@pytest.mark.parametrize("induced", [True, False])
def test_compile_matches_oracle(lib, induced):
    for a in _all_patterns():
        s = gz.compile_pattern(a, induced)
        info = s.info()
        best, cost = P.pick_schedule(a, induced)
        assert info["order"] == tuple(best)
        assert info["bound"] == P.reduced_bounds(a, best)
        assert info["aut_size"] == P.multiplicity(a)
        assert info["n_distinct"] == len(P.distinct_schedules(a))
        assert info["cost"] == pytest.approx(cost, rel=1e-13)


def test_enumeration_matches_explorer(lib):
    for a in _all_patterns():
        got = gz.enumerate_schedules(a, True)
        want = P.distinct_schedules(a)
        assert [o for o, _ in got] == [tuple(s) for s in want]
        for (o, c) in got:
            assert c == pytest.approx(P.analytic_cost(a, o, True), rel=1e-13)


def test_fixed_order_bounds_match_oracle(lib):
    for a in _all_patterns():
        for s in P.valid_schedules_bruteforce(a)[:40]:
            info = gz.compile_pattern_order(a, s, True).info()
            assert info["order"] == tuple(s)
            assert info["bound"] == P.reduced_bounds(a, s)


def test_no_restrict_flag_drops_bounds(lib):
    s = gz.compile_pattern(P.named("k4"), True, gz.SCHED_NO_RESTRICT)
    assert s.info()["bound"] == [-1, -1, -1, -1]


def test_k8_pattern_compiles(lib):
    a = P.named("c8")
    info = gz.compile_pattern(a, True).info()
    assert info["aut_size"] == 16
    assert len(info["order"]) == 8


@pytest.mark.parametrize("bad", ["disconnected", "selfloop", "asym", "k1", "k9", "entry2"])
def test_bad_patterns_rejected(lib, bad):
    if bad == "disconnected":
        a = np.zeros((4, 4), np.uint8)
        a[0, 1] = a[1, 0] = a[2, 3] = a[3, 2] = 1
    elif bad == "selfloop":
        a = np.array(P.named("triangle"), np.uint8)
        a[1, 1] = 1
    elif bad == "asym":
        a = np.array(P.named("c4"), np.uint8)
        a[0, 2] = 1
    elif bad == "k1":
        a = np.zeros((1, 1), np.uint8)
    elif bad == "k9":
        a = np.array(P.named("c9") if False else np.ones((9, 9), np.uint8) - np.eye(9, dtype=np.uint8))
    else:
        a = np.array(P.named("triangle"), np.uint8) * 2
    with pytest.raises(gz.GzError) as e:
        gz.compile_pattern(a, True)
    assert e.value.status == gz.GZ_EINVAL


def test_invalid_order_rejected(lib):
    with pytest.raises(gz.GzError) as e:
        gz.compile_pattern_order(P.named("p4"), (0, 2, 1, 3), True)  # 2 not adjacent to 0
    assert e.value.status == gz.GZ_EINVAL
    with pytest.raises(gz.GzError):
        gz.compile_pattern_order(P.named("p4"), (0, 1, 1, 3), True)  # not a permutation


def test_null_handles_rejected(lib):
    import ctypes
    out = ctypes.c_uint64()
    assert lib.gz_count(None, None, None, ctypes.byref(out)) == gz.GZ_EINVAL
    assert lib.gz_count_roots(None, None, None, 0, None, None) == gz.GZ_EINVAL
    assert lib.gz_count_bytes(None, None, None, None, None) == gz.GZ_EINVAL
    assert lib.gz_graph_info(None, None, None, None, None) == gz.GZ_EINVAL
    assert lib.gz_schedule_info(None, None, None, None, None, None) == gz.GZ_EINVAL
    assert gz.status_string(gz.GZ_EOVERFLOW) == "count overflows 64 bits"
    lib.gz_free_graph(None)
    lib.gz_free_schedule(None)


# ------------------------------------------------------------ graph prep


def _oracle_prep(e, reindex=True):
    g = oracle.from_edge_tuple(e, reindex)
    return g.rowptr.astype(np.int32), g.col, g.new_of_old, oracle.lo_end(g)


@pytest.mark.parametrize("which", ["er", "rmat", "cl", "star", "empty", "loops"])
def test_prepare_matches_oracle(lib, which):
    if which == "er":
        e = synth.er_edges(300, 0.05, 3)
    elif which == "rmat":
        e = synth.rmat_edges(12, 8, seed=4)
    elif which == "cl":
        e = synth.chung_lu_edges(3000, 2.2, 12.0, 5, cap=False)
    elif which == "star":
        e = synth.star_edges(20)
    elif which == "empty":
        e = (np.zeros(0, np.int32), np.zeros(0, np.int32), 7)
    else:
        e = (np.array([0, 1, 1, 2, 2, 3], np.int32), np.array([0, 2, 2, 1, 3, 3], np.int32), 5)
    for reindex in (True, False):
        r, c, perm, lo = gz.prepare_edges(*e, flags=0 if reindex else gz.GRAPH_NO_REINDEX)
        orr, oc, onew, olo = _oracle_prep(e, reindex)
        assert np.array_equal(r, orr)
        assert np.array_equal(c, oc)
        assert np.array_equal(lo, olo)
        # library returns old_of_new, the oracle new_of_old
        assert np.array_equal(onew[perm], np.arange(e[2]))


def test_prepare_rejects_bad_endpoints(lib):
    with pytest.raises(gz.GzError) as e:
        gz.prepare_edges(np.array([0, 5], np.int32), np.array([1, 2], np.int32), 4)
    assert e.value.status == gz.GZ_EINVAL
    with pytest.raises(gz.GzError):
        gz.prepare_edges(np.array([-1], np.int32), np.array([1], np.int32), 4)
