"""GPU parity of the neighbour bitmaps of high-degree vertices.

The generic path answers a membership probe into the list of a hub (one of
the leading vertices of degree >= GZ_HUB_MIN_DEG after the degree reindex)
with one bit of that hub's bitmap instead of a binary search.  The default
threshold leaves the small test graphs without hubs, so these tests force it
low (down to every vertex being a hub), cap the bitmaps' memory so that only
part of the leading run gets rows, switch them off, and combine them with
the two-phase split and forced inclusion-exclusion.  Counts must stay
bit-exact against the oracle, in total and per root.

Last-loop items whose walk reaches GZ_LONG_MIN elements are counted by the
whole wave, merging probe lists up to GZ_MERGE_RATIO times the walk's length
through an LDS window and probing longer ones per element; both are forced
to their extremes here (every item long; every list merged, or none).

Groups of last-loop items that walk their own rows may instead be swept: the
earlier loops' lists become one LDS bit mask per block of 2^15 vertex ids
(hub bitmaps ANDed, negative lists without a bitmap clearing their entries).
GZ_SWEEP_MIN=1 sweeps every eligible group; a copy of the test graph with its
ids spread over 150,000 (no degree reindex) makes the rows span several
blocks, with hub and non-hub lists, split and unsplit loops, and either
choice against inclusion-exclusion (GZ_SWEEP_IE)."""

import os
import sys

import numpy as np
import pytest

import oracle
from oracle import patterns as P
from paper_1911_12877_amd import gz, synth

pytestmark = pytest.mark.gpu

ENV = ("GZ_HUB_MIN_DEG", "GZ_HUB_MAX_KB", "GZ_SPLIT_MIN_LEN", "GZ_IE_FORCE", "GZ_LONG_MIN",
       "GZ_MERGE_RATIO", "GZ_SWEEP_MIN", "GZ_SWEEP_IE")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gz.library()
    yield
    for k in ENV:
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


PATS = [(nm, ind) for nm in ("triangle", "c4", "diamond", "tailed_triangle", "house", "k5e",
                             "c5", "k4", "p4", "star4") for ind in (True, False)] + \
    [("c6chord03", True), ("k6e", True)]


@pytest.fixture(scope="module")
def cl_case():
    e = synth.chung_lu_edges(1500, 2.2, 10.0, 71, cap=False)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    want = {(nm, ind): oracle.count(O, P.named(nm), ind) for nm, ind in PATS}
    return G, O, want


# (min degree, cap in KiB): every vertex, the hubs of degree >= 8 or 64,
# and a cap that cuts the leading run after a few rows (1500-vertex rows
# take 188 bytes)
SETTINGS = [(1, None), (8, None), (64, None), (1, 1), ("1", 0)]


@pytest.mark.parametrize("setting", SETTINGS)
def test_hubs_match_oracle(cl_case, setting):
    G, _, want = cl_case
    md, cap = setting
    kv = {"GZ_HUB_MIN_DEG": md}
    if cap is not None:
        kv["GZ_HUB_MAX_KB"] = cap
    for nm, induced in PATS:
        s = gz.compile_pattern(P.named(nm), induced)
        with _env(**kv):
            _say("hubs", setting, nm, induced)
            got = gz.count(G, s)
        assert got == want[(nm, induced)], (nm, induced, setting)


def test_hubs_with_split_and_inclusion_exclusion(cl_case):
    G, _, want = cl_case
    for nm, induced in PATS:
        s = gz.compile_pattern(P.named(nm), induced)
        for kv in ({"GZ_HUB_MIN_DEG": 4, "GZ_SPLIT_MIN_LEN": 0},
                   {"GZ_HUB_MIN_DEG": 4, "GZ_IE_FORCE": 1},
                   {"GZ_HUB_MIN_DEG": 4, "GZ_IE_FORCE": 1, "GZ_SPLIT_MIN_LEN": 0}):
            with _env(**kv):
                got = gz.count(G, s)
            assert got == want[(nm, induced)], (nm, induced, kv)


@pytest.mark.parametrize("nm", ["c4", "house", "tailed_triangle", "k5e"])
def test_hubs_per_root(nm):
    e = synth.rmat_edges(10, 8, seed=72)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    pat = P.named(nm)
    s = gz.compile_pattern(pat, True)
    roots = np.arange(O.n, dtype=np.int32)
    total, want = oracle.count(O, pat, True, order=s.info()["order"], relations="thm2",
                               roots=roots, per_root=True)
    with _env(GZ_HUB_MIN_DEG=16):
        got = gz.count_roots(G, s, roots)
    assert np.array_equal(got, want)
    assert int(got.astype(object).sum()) == total


def test_hubs_every_small_pattern():
    graphs = [synth.er_edges(14, 0.45, 73), synth.rmat_edges(6, 6, seed=74),
              synth.chung_lu_edges(40, 2.3, 6.0, 75, cap=False), synth.star_edges(9)]
    for e in graphs:
        G = gz.load_edges(*e)
        O = oracle.from_edge_tuple(e)
        for k in (3, 4, 5):
            for pat in P.connected_patterns(k):
                for induced in (True, False):
                    want = oracle.count(O, pat, induced)
                    s = gz.compile_pattern(pat, induced)
                    with _env(GZ_HUB_MIN_DEG=1):
                        assert gz.count(G, s) == want, (k, pat, induced)


def test_hubs_without_reindex():
    """Orientation off: ids keep the input order, so only the leading run of
    high-degree ids gets rows (a star whose hub is vertex 0, then the rest)."""
    a, b, n = synth.star_edges(60)
    na, nb, _ = synth.er_edges(n, 0.08, 76)
    e = (np.concatenate([a, na]).astype(np.int32), np.concatenate([b, nb]).astype(np.int32), n)
    G = gz.load_edges(*e, flags=gz.GRAPH_NO_REINDEX)
    O = oracle.from_edge_tuple(e, reindex_by_degree=False)
    for nm in ("c4", "diamond", "tailed_triangle", "house"):
        pat = P.named(nm)
        want = oracle.count(O, pat, True)
        with _env(GZ_HUB_MIN_DEG=5):
            assert gz.count(G, gz.compile_pattern(pat, True)) == want, nm


# (long-walk threshold, merge ratio, hub threshold): every item walked by the
# whole wave with every list merged, with none merged (all probed, by bitmap
# or binary search), and a middle setting; plus forced inclusion-exclusion
LONG = [(1, 1 << 20, 1024), (1, 0, 4), (1, 0, 1024), (16, 2, 8)]


@pytest.mark.parametrize("setting", LONG)
def test_long_walks_match_oracle(cl_case, setting):
    G, _, want = cl_case
    lm, ratio, hub = setting
    for nm, induced in PATS:
        s = gz.compile_pattern(P.named(nm), induced)
        for extra in ({}, {"GZ_IE_FORCE": 1}, {"GZ_SPLIT_MIN_LEN": 0}):
            with _env(GZ_LONG_MIN=lm, GZ_MERGE_RATIO=ratio, GZ_HUB_MIN_DEG=hub, **extra):
                _say("long", setting, extra, nm, induced)
                got = gz.count(G, s)
            assert got == want[(nm, induced)], (nm, induced, setting, extra)


def test_long_walks_every_small_pattern():
    graphs = [synth.er_edges(14, 0.45, 81), synth.rmat_edges(6, 6, seed=82),
              synth.chung_lu_edges(60, 2.2, 8.0, 83, cap=False)]
    for e in graphs:
        G = gz.load_edges(*e)
        O = oracle.from_edge_tuple(e)
        for k in (3, 4, 5):
            for pat in P.connected_patterns(k):
                for induced in (True, False):
                    want = oracle.count(O, pat, induced)
                    s = gz.compile_pattern(pat, induced)
                    for ratio in (0, 1 << 20):
                        with _env(GZ_LONG_MIN=1, GZ_MERGE_RATIO=ratio):
                            assert gz.count(G, s) == want, (k, pat, induced, ratio)


@pytest.mark.parametrize("nm", ["tailed_triangle", "c4", "k5e"])
def test_long_walks_per_root(nm):
    e = synth.rmat_edges(10, 8, seed=84)
    G = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    pat = P.named(nm)
    s = gz.compile_pattern(pat, True)
    roots = np.arange(O.n, dtype=np.int32)
    _, want = oracle.count(O, pat, True, order=s.info()["order"], relations="thm2",
                           roots=roots, per_root=True)
    with _env(GZ_LONG_MIN=8, GZ_MERGE_RATIO=3, GZ_HUB_MIN_DEG=16):
        got = gz.count_roots(G, s, roots)
    assert np.array_equal(got, want)


# ------------------------------------------------------------------ sweep

SWEEP = [  # (hub threshold, hub cap KiB, sweep_ie, extra)
    (1, None, 1 << 20, {}),
    (1, None, 0, {}),
    (8, None, 8, {"GZ_SPLIT_MIN_LEN": 0}),
    (1, 0, 1 << 20, {}),
    (1, 1, 8, {"GZ_LONG_MIN": 1}),
]


@pytest.mark.parametrize("setting", SWEEP)
def test_sweep_one_block(cl_case, setting):
    G, _, want = cl_case
    hub, cap, ie, extra = setting
    kv = dict(GZ_SWEEP_MIN=1, GZ_SWEEP_IE=ie, GZ_HUB_MIN_DEG=hub, **extra)
    if cap is not None:
        kv["GZ_HUB_MAX_KB"] = cap
    for nm, induced in PATS:
        s = gz.compile_pattern(P.named(nm), induced)
        with _env(**kv):
            _say("sweep", setting, nm, induced)
            got = gz.count(G, s)
        assert got == want[(nm, induced)], (nm, induced, setting)


SPREAD_N = 150000


def spread_edges(seed=71):
    """The Chung-Lu test graph relabelled: its 32 highest-degree vertices at
    ids 0..31 (the leading run that gets bitmaps), the others at seeded
    random ids up to SPREAD_N, in no degree order."""
    src, dst, n = synth.chung_lu_edges(1500, 2.2, 10.0, seed, cap=False)
    deg = np.bincount(np.concatenate([src, dst]), minlength=n)
    by_deg = np.argsort(-deg, kind="stable")
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    rest = rng.choice(np.arange(32, SPREAD_N), size=n - 32, replace=False)
    new = np.empty(n, dtype=np.int64)
    new[by_deg[:32]] = np.arange(32)
    new[by_deg[32:]] = rest
    return new[src].astype(np.int32), new[dst].astype(np.int32), SPREAD_N


@pytest.fixture(scope="module")
def spread_case(cl_case):
    _, _, want = cl_case  # totals do not depend on the labels
    e = spread_edges()
    G = gz.load_edges(*e, flags=gz.GRAPH_NO_REINDEX)
    return G, e, want


@pytest.mark.parametrize("setting", SWEEP)
def test_sweep_several_blocks(spread_case, setting):
    G, _, want = spread_case
    hub, cap, ie, extra = setting
    kv = dict(GZ_SWEEP_MIN=1, GZ_SWEEP_IE=ie, GZ_HUB_MIN_DEG=hub, **extra)
    if cap is not None:
        kv["GZ_HUB_MAX_KB"] = cap
    for nm, induced in PATS:
        s = gz.compile_pattern(P.named(nm), induced)
        with _env(**kv):
            _say("sweep spread", setting, nm, induced)
            got = gz.count(G, s)
        assert got == want[(nm, induced)], (nm, induced, setting)


@pytest.mark.parametrize("nm", ["tailed_triangle", "c4", "diamond", "house"])
def test_sweep_several_blocks_per_root(spread_case, nm):
    G, e, _ = spread_case
    O = oracle.from_edge_tuple(e, reindex_by_degree=False)
    pat = P.named(nm)
    s = gz.compile_pattern(pat, True)
    roots = np.unique(np.concatenate([e[0], e[1]])).astype(np.int32)
    total, want = oracle.count(O, pat, True, order=s.info()["order"], relations="thm2",
                               roots=roots, per_root=True)
    with _env(GZ_SWEEP_MIN=1, GZ_HUB_MIN_DEG=1):
        got = gz.count_roots(G, s, roots)
    assert np.array_equal(got, want)
    assert int(got.astype(object).sum()) == total
