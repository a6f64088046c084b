"""GPU graph preparation (GZ_GRAPH_PREP_DEVICE): normalisation and degree
reindex by device radix sorts must give exactly the arrays of the oracle's
normalisation and reindex (Section 6, first technique) and of the host path,
for inputs with self-loops, duplicates, both orientations, isolated vertices
and empty edge lists, from host or device input arrays; counts on the
prepared graph match."""

import sys
import time

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


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _cases():
    yield "er300", synth.er_edges(300, 0.05, 71)
    yield "rmat12", synth.rmat_edges(12, 16, seed=72)
    yield "cl5000", synth.chung_lu_edges(5000, 2.2, 12.0, 73, cap=False)
    yield "star40", synth.star_edges(40)
    yield "k12", synth.complete_edges(12)
    # self-loops, duplicates, both orientations, isolated vertices 7..9
    yield "messy", (np.array([0, 1, 1, 2, 3, 3, 5, 6, 0, 4], np.int32),
                    np.array([1, 0, 1, 3, 2, 3, 6, 5, 1, 4], np.int32), 10)
    yield "no_edges", (np.zeros(0, np.int32), np.zeros(0, np.int32), 6)
    yield "loops_only", (np.array([0, 1, 2], np.int32), np.array([0, 1, 2], np.int32), 3)
    yield "one_vertex", (np.zeros(0, np.int32), np.zeros(0, np.int32), 1)


@pytest.mark.parametrize("name", [c[0] for c in _cases()])
def test_device_prep_matches_oracle_and_host(name):
    e = dict(_cases())[name]
    Gd = gz.load_edges(*e, flags=gz.GRAPH_PREP_DEVICE)
    Gh = gz.load_edges(*e)
    O = oracle.from_edge_tuple(e)
    rd, cd, od = gz.graph_export(Gd)
    rh, ch, oh = gz.graph_export(Gh)
    assert np.array_equal(rd, O.rowptr.astype(np.int32)), name
    assert np.array_equal(cd, O.col), name
    assert np.array_equal(O.new_of_old[od], np.arange(O.n)), name
    assert np.array_equal(rd, rh) and np.array_equal(cd, ch) and np.array_equal(od, oh)
    assert Gd.info() == Gh.info()
    for nm in ("triangle", "k4", "tailed_triangle", "c4"):
        s = gz.compile_pattern(P.named(nm), True)
        assert gz.count(Gd, s) == gz.count(Gh, s), (name, nm)


def test_device_prep_without_reindex_and_device_inputs():
    import torch
    e = synth.rmat_edges(11, 8, seed=74)
    Gh = gz.load_edges(*e, flags=gz.GRAPH_NO_REINDEX)
    Gd = gz.load_edges(*e, flags=gz.GRAPH_NO_REINDEX | gz.GRAPH_PREP_DEVICE)
    for a, b in zip(gz.graph_export(Gh), gz.graph_export(Gd)):
        assert np.array_equal(a, b)
    src = torch.from_numpy(e[0]).cuda()
    dst = torch.from_numpy(e[1]).cuda()
    Gt = gz.load_edges(src, dst, e[2], flags=gz.GRAPH_PREP_DEVICE)
    Gr = gz.load_edges(*e)
    for a, b in zip(gz.graph_export(Gr), gz.graph_export(Gt)):
        assert np.array_equal(a, b)
    s = gz.compile_pattern(P.named("k4"), True)
    assert gz.count(Gt, s) == gz.count(Gr, s) == gz.count(Gd, s)


def test_device_prep_rejects_bad_endpoints():
    for src, dst, n in (([0, 5], [1, 2], 5), ([0, -1], [1, 2], 5), ([0], [1], 0)):
        with pytest.raises(gz.GzError) as ex:
            gz.load_edges(np.array(src, np.int32), np.array(dst, np.int32), n,
                          flags=gz.GRAPH_PREP_DEVICE)
        assert ex.value.status == gz.GZ_EINVAL


def test_device_prep_rmat20_full_size():
    """R-MAT scale 20 (33.5M samples): the device arrays equal the host
    preparation's entry by entry; timings of both are printed."""
    import torch
    e = synth.config_graph("rmat20")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Gh = gz.load_edges(*e)
    th = time.perf_counter() - t0
    t0 = time.perf_counter()
    Gd = gz.load_edges(*e, flags=gz.GRAPH_PREP_DEVICE)
    td = time.perf_counter() - t0
    _say(f"rmat20 preparation: host {th:.3f} s, device {td:.3f} s (with host copies)")
    for a, b in zip(gz.graph_export(Gh), gz.graph_export(Gd)):
        assert np.array_equal(a, b)
    assert Gd.info() == Gh.info()
    s = gz.compile_pattern(P.named("k4"), True)
    assert gz.count(Gd, s) == gz.count(Gh, s)
