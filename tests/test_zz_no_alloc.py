"""gz_count_noalloc (the count for callers that cannot allocate device
memory) against gz_count through the C-ABI: the same exact counts, on two
calls in a row of which the second has the smaller input, on graphs
prepared on the host and on the device, with and without hub bitmaps and
whole-wave walks, and where long loop bases are expanded in place."""

import os

import numpy as np
import pytest

from paper_1911_12877_amd import gz, synth
from oracle import patterns as P

pytestmark = pytest.mark.gpu

PATS = [("triangle", True), ("c4", True), ("diamond", True), ("tailed_triangle", True),
        ("house", True), ("k4", True), ("k5e", True), ("c4", False), ("c6chord03", True)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gz.library()
    yield
    for k in ("GZ_HUB_MIN_DEG", "GZ_LONG_MIN"):
        os.environ.pop(k, None)


def _pair(big, small):
    """Counts of every pattern, large graph then small graph, by both entry
    points."""
    for nm, induced in PATS:
        s = gz.compile_pattern(P.named(nm), induced)
        for G in (big, small):
            want = gz.count(G, s)
            got = gz.count_noalloc(G, s)
            assert got == want, (nm, induced, G.info()["n"])


def test_noalloc_matches_count_large_then_small():
    big = gz.load_edges(*synth.chung_lu_edges(3000, 2.2, 10.0, 91, cap=False))
    small = gz.load_edges(*synth.er_edges(300, 0.05, 92))
    _pair(big, small)


def test_noalloc_device_prepared_graphs():
    big = gz.load_edges(*synth.rmat_edges(11, 8, seed=93), flags=gz.GRAPH_PREP_DEVICE)
    small = gz.load_edges(*synth.rmat_edges(7, 8, seed=94), flags=gz.GRAPH_PREP_DEVICE)
    _pair(big, small)


def test_noalloc_with_hubs_and_long_walks():
    """After a gz_count built the hub bitmaps (low threshold), the
    allocation-free count uses them; every last-loop item walked by the
    whole wave as well."""
    os.environ["GZ_HUB_MIN_DEG"] = "8"
    os.environ["GZ_LONG_MIN"] = "1"
    try:
        big = gz.load_edges(*synth.chung_lu_edges(2000, 2.1, 12.0, 95, cap=False))
        small = gz.load_edges(*synth.star_edges(50))
        _pair(big, small)
    finally:
        os.environ.pop("GZ_HUB_MIN_DEG", None)
        os.environ.pop("GZ_LONG_MIN", None)


def test_noalloc_two_hubs_bases_expanded_in_place():
    """Leaves above id 2048 meet hub lists longer than the split threshold:
    gz_count records and splits them, the allocation-free count expands them
    in place; the counts agree."""
    a, b, n = synth.complete_bipartite_edges(2, 3000)
    na, nb, _ = synth.er_edges(n, 4.0 / n, 96)
    e = (np.concatenate([a, na]).astype(np.int32), np.concatenate([b, nb]).astype(np.int32), n)
    big = gz.load_edges(*e)
    small = gz.load_edges(*synth.cycle_edges(40))
    _pair(big, small)


def test_noalloc_empty_graph():
    G = gz.load_edges(np.zeros(0, np.int32), np.zeros(0, np.int32), 5)
    s = gz.compile_pattern(P.named("triangle"), True)
    assert gz.count_noalloc(G, s) == 0 == gz.count(G, s)
