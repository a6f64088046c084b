"""GPU parity of the generic path's alternative evaluations.

Two-phase split: prefixes whose loop base is long are recorded by the first
launch and expanded in pieces by a second.  The threshold and the
record-list capacity are forced low so that almost every prefix takes the
second phase, or the list overflows and the rest are expanded in place; a
two-hub graph exercises the default threshold.

Inclusion-exclusion in the last loop: forced for every item that has
negative lists (GZ_IE_FORCE=1), on every pattern of up to 5 vertices and on
larger ones; the two-hub graph takes it by itself for hub-rooted tails.

Counts must stay bit-exact against the oracle, in total and per root."""

import os
import sys

import numpy as np
import pytest

import oracle
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
    for k in ("GZ_SPLIT_MIN_LEN", "GZ_SPLIT_CAP", "GZ_IE_FORCE"):
        os.environ.pop(k, None)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


class _env:
    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        for k, v in self.kv.items():
            os.environ[k] = str(v)

    def __exit__(self, *exc):
        for k in self.kv:
            os.environ.pop(k, None)


def _two_hubs(m, seed):
    """Two hubs joined to the same m leaves, plus sparse noise among leaves."""
    a, b, n = synth.complete_bipartite_edges(2, m)
    na, nb, _ = synth.er_edges(n, 4.0 / n, seed)
    return np.concatenate([a, na]).astype(np.int32), np.concatenate([b, nb]).astype(np.int32), n


PATS = [(nm, ind) for nm in ("c4", "diamond", "tailed_triangle", "house", "k5e", "c5", "k4",
                             "k6e") for ind in (True, False)] + [("c6chord03", True)]


@pytest.fixture(scope="module")
def cl_case():
    e = synth.chung_lu_edges(1500, 2.2, 10.0, 51, cap=False)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    want = {(nm, ind): oracle.count(O, P.named(nm), ind) for nm, ind in PATS}
    return G, want


@pytest.mark.parametrize("split", [(0, None), (64, None), (0, 1), (0, 37)])
def test_forced_split_matches_oracle(cl_case, split):
    G, want = cl_case
    min_len, cap = split
    kv = {"GZ_SPLIT_MIN_LEN": min_len}
    if cap is not None:
        kv["GZ_SPLIT_CAP"] = cap
    for nm, induced in PATS:
        s = gz.compile_pattern(P.named(nm), induced)
        with _env(**kv):
            _say("split", split, nm, induced)
            got = gz.count(G, s)
        assert got == want[(nm, induced)], (nm, induced, split)


@pytest.mark.parametrize("nm", ["house", "c4", "k5e"])
def test_forced_split_per_root(nm):
    e = synth.rmat_edges(10, 8, seed=52)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    pat = P.named(nm)
    s = gz.compile_pattern(pat, True)
    roots = np.arange(O.n, dtype=np.int32)
    total, want = oracle.count(O, pat, True, order=s.info()["order"], relations="thm2",
                               roots=roots, per_root=True)
    with _env(GZ_SPLIT_MIN_LEN=0):
        got = gz.count_roots(G, s, roots)
        sub = np.array([5, 5, 0, O.n - 1, 17, 3], np.int32)
        got_sub = gz.count_roots(G, s, sub)
    assert np.array_equal(got, want)
    assert np.array_equal(got_sub, want[sub])
    assert int(got.astype(object).sum()) == total


@pytest.fixture(scope="module")
def hub_case():
    e = _two_hubs(3000, 53)
    return gz.load_edges(*e), oracle.from_edge_tuple(e)


@pytest.mark.parametrize("nm", ["c4", "diamond", "house", "tailed_triangle"])
def test_two_hubs_default_threshold(hub_case, nm):
    """Leaves of ids above 2048 meet hub lists longer than the default
    threshold in loop 2, so the second phase runs without any override."""
    G, O = hub_case
    pat = P.named(nm)
    for induced in (True, False):
        _say("two hubs", nm, induced)
        want = oracle.count(O, pat, induced)
        s = gz.compile_pattern(pat, induced)
        assert gz.count(G, s) == want, (nm, induced)
        # the same count with splitting switched off (threshold above any base)
        with _env(GZ_SPLIT_MIN_LEN=1 << 30):
            assert gz.count(G, s) == want, (nm, induced)


def test_forced_inclusion_exclusion_small_patterns():
    graphs = [synth.er_edges(14, 0.45, 61), synth.rmat_edges(6, 6, seed=62),
              synth.chung_lu_edges(40, 2.3, 6.0, 63, cap=False), synth.star_edges(9)]
    for e in graphs:
        G = gz.load_edges(*e)
        O = oracle.from_edge_tuple(e)
        for k in (3, 4, 5):
            for pat in P.connected_patterns(k):
                want = oracle.count(O, pat, True)
                s = gz.compile_pattern(pat, True)
                with _env(GZ_IE_FORCE=1):
                    assert gz.count(G, s) == want, (k, pat)


def test_forced_inclusion_exclusion_medium(cl_case):
    G, want = cl_case
    for nm, induced in PATS:
        s = gz.compile_pattern(P.named(nm), induced)
        with _env(GZ_IE_FORCE=1):
            _say("ie", nm, induced)
            assert gz.count(G, s) == want[(nm, induced)], (nm, induced)
        with _env(GZ_IE_FORCE=1, GZ_SPLIT_MIN_LEN=0):
            assert gz.count(G, s) == want[(nm, induced)], (nm, induced, "split")


@pytest.mark.parametrize("nm", ["house", "tailed_triangle", "c6chord02"])
def test_forced_inclusion_exclusion_per_root(nm):
    e = synth.rmat_edges(9, 8, seed=64)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    pat = P.named(nm)
    s = gz.compile_pattern(pat, True)
    roots = np.arange(O.n, dtype=np.int32)
    _, want = oracle.count(O, pat, True, order=s.info()["order"], relations="thm2",
                           roots=roots, per_root=True)
    with _env(GZ_IE_FORCE=1):
        got = gz.count_roots(G, s, roots)
    assert np.array_equal(got, want)
    # with every prefix split as well
    with _env(GZ_IE_FORCE=1, GZ_SPLIT_MIN_LEN=0):
        got = gz.count_roots(G, s, roots)
    assert np.array_equal(got, want)


def test_larger_patterns_forced_inclusion_exclusion():
    e = synth.er_edges(13, 0.6, 65)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    for nm in ("c6", "c6chord03", "k6e", "c7", "k7e", "p6", "c8"):
        pat = P.named(nm)
        want = oracle.count(O, pat, True)
        with _env(GZ_IE_FORCE=1):
            assert gz.count(G, gz.compile_pattern(pat, True)) == want, nm


def test_invalid_overrides_ignored():
    e = synth.er_edges(300, 0.05, 54)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    pat = P.named("house")
    s = gz.compile_pattern(pat, True)
    want = oracle.count(O, pat, True)
    for bad in ("-3", "abc", "12x", ""):
        with _env(GZ_SPLIT_MIN_LEN=bad, GZ_SPLIT_CAP=bad):
            assert gz.count(G, s) == want, bad
