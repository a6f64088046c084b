"""Pins of the oracle's compile-side algorithms (automorphisms, Algorithm 1,
Theorem 2, Algorithms 2 and 3, the performance model, motif enumeration)
against the paper's worked examples and closed forms."""

import itertools
import math

import pytest

from oracle import patterns as P


def _adj(entry):
    return P.from_edges(entry["k"], [tuple(e) for e in entry["edges"]])


# ------------------------------------------------------- worked examples


def test_rectangle_relations(golden):
    g = golden["rectangle"]
    a = _adj(g)
    s = tuple(g["schedule"])
    rel = P.restrictions(a, s)
    assert sorted(rel) == sorted(tuple(r) for r in g["relations"])
    assert P.reduced_bounds(a, s) == g["reduced_bound_by_position"]
    assert P.multiplicity(a) == g["multiplicity"]


def test_rectangle_pass_rate(golden):
    g = golden["rectangle"]
    a = _adj(g)
    b = P.reduced_bounds(a, tuple(g["schedule"]))
    assert P.forest_pass_rate(b, 3) == pytest.approx(g["pass_rate_last_level"], abs=0)
    # per-level pass rates of the nested integral: 1, 1/2, 1/6, 1/8
    assert [P.forest_pass_rate(b, i) for i in range(4)] == \
        pytest.approx([1.0, 0.5, 1.0 / 6.0, 0.125], rel=1e-15)


def test_tailed_triangle_equivalence(golden):
    g = golden["tailed_triangle"]
    a = _adj(g)
    s1, s2 = (tuple(s) for s in g["equivalent_schedules"])
    assert any(tuple(x[v] for v in s1) == s2 for x in P.automorphisms(a))
    ds = P.distinct_schedules(a)
    assert (s1 in ds) != (s2 in ds)  # exactly one of the pair is emitted


def test_paper_multiplicities(golden):
    g = golden["multiplicities"]
    assert P.multiplicity(P.named("k7e")) == g["k7_minus_edge"]
    assert P.multiplicity(P.named("c5")) == g["pentagon"]


def test_motif_pattern_counts(golden):
    g = golden["motif_pattern_counts"]
    assert len(P.connected_patterns(3)) == g["3"]
    assert len(P.connected_patterns(4)) == 6   # textbook value
    assert len(P.connected_patterns(5)) == g["5"]


# --------------------------------------------------------- closed forms


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_aut_closed_forms(k):
    assert P.multiplicity(P.named(f"k{k}")) == math.factorial(k)
    assert P.multiplicity(P.named(f"c{k}")) == 2 * k
    assert P.multiplicity(P.named(f"p{k}")) == 2
    assert P.multiplicity(P.named(f"star{k}")) == math.factorial(k - 1)
    if k >= 4:
        assert P.multiplicity(P.named(f"k{k}e")) == 2 * math.factorial(k - 2)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_schedule_space_closed_forms(k, golden):
    kk = P.named(f"k{k}")
    assert len(P.valid_schedules_bruteforce(kk)) == math.factorial(k)
    assert len(P.distinct_schedules(kk)) == golden["schedule_space"]["clique_distinct"]
    path = P.named(f"p{k}")
    assert len(P.distinct_schedules(path)) == 2 ** (k - 2)
    assert len(P.valid_schedules_bruteforce(path)) == 2 ** (k - 1)
    cyc = P.named(f"c{k}")
    assert len(P.valid_schedules_bruteforce(cyc)) == k * 2 ** (k - 2)
    assert len(P.distinct_schedules(cyc)) == 2 ** (k - 3)
    st = P.named(f"star{k}")
    assert len(P.valid_schedules_bruteforce(st)) == 2 * math.factorial(k - 1)
    assert len(P.distinct_schedules(st)) == 2
    if k >= 4:
        ke = P.named(f"k{k}e")
        assert len(P.valid_schedules_bruteforce(ke)) == \
            math.factorial(k) - 2 * math.factorial(k - 2)
        assert len(P.distinct_schedules(ke)) == math.comb(k, 2) - 1


def _all_patterns(kmax):
    for k in range(2, kmax + 1):
        for a in P.connected_patterns(k):
            yield k, a


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_explorer_theorem3(k):
    """Algorithm 3 emits one schedule per equivalence class: #distinct equals
    #valid / |Aut|, every emitted schedule is valid, no two are equivalent,
    and every valid schedule is equivalent to an emitted one."""
    for a in P.connected_patterns(k):
        auts = P.automorphisms(a)
        valid = P.valid_schedules_bruteforce(a)
        assert sorted(valid) == sorted(P.valid_schedules_recursive(a))
        ds = P.distinct_schedules(a)
        assert len(ds) * len(auts) == len(valid)
        assert all(P.is_valid_schedule(a, s) for s in ds)
        classes = set()
        for s in ds:
            cls = frozenset(tuple(x[v] for v in s) for x in auts)
            assert not (cls & classes)
            classes |= cls
        assert classes == set(valid)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_restriction_product_equals_multiplicity(k):
    """Appendix closing remark: at the bottom loop the pass rate is
    1/multiplicity, for every pattern and every valid schedule."""
    for a in P.connected_patterns(k):
        m = P.multiplicity(a)
        for s in P.distinct_schedules(a):
            assert P.restricted_pass_product(a, s) == m


def test_restriction_product_larger_patterns():
    for name in ["k6e", "k7e", "c6chord03", "c6chord02", "house", "c6"]:
        a = P.named(name)
        m = P.multiplicity(a)
        for s in P.distinct_schedules(a):
            assert P.restricted_pass_product(a, s) == m


def test_relations_point_forward():
    """Theorem 2's proof: every relation (S[a], S[b]) has a < b."""
    for k, a in _all_patterns(5):
        for s in P.distinct_schedules(a):
            for x, y in P.relations_as_positions(a, s):
                assert x < y


def test_thm2_bounds_keep_latest_relation():
    """The reduced bound of each position is the latest earlier position
    related to it, and the map form of the algorithm (overwrite x(v) <- v in
    schedule order) gives the same result."""
    for k, a in _all_patterns(5):
        for s in P.distinct_schedules(a):
            pos = {v: i for i, v in enumerate(s)}
            m = {}
            group = P.automorphisms(a)
            for v in s:
                keep = []
                for x in group:
                    if x[v] == v:
                        keep.append(x)
                    else:
                        m[x[v]] = v
                group = keep
            expect = [pos[m[v]] if v in m else -1 for v in s]
            assert P.reduced_bounds(a, s) == expect


def test_analytic_cost_model_orders_tailed_triangle(golden):
    """Section 5.1: [C,D,B,A] (per triangle) should be cheaper than
    [A,B,C,D] (per wedge)."""
    a = _adj(golden["tailed_triangle"])
    per_wedge = P.analytic_cost(a, (0, 1, 2, 3), induced=True)
    per_triangle = P.analytic_cost(a, (2, 3, 1, 0), induced=True)
    assert per_triangle < per_wedge


def test_analytic_cost_clique_closed_form():
    """K_k, identity schedule, chain of bounds: cost = sum_i n^(i+1)
    p^(i(i+1)/2) / (i+1)! with p = 5/999 and n = 1000."""
    n, p = 1000, 5.0 / 999
    for k in (3, 4, 5):
        a = P.named(f"k{k}")
        want = sum(n ** (i + 1) * p ** (i * (i + 1) // 2) / math.factorial(i + 1)
                   for i in range(k))
        assert P.analytic_cost(a, tuple(range(k)), True) == pytest.approx(want, rel=1e-12)


def test_pick_is_a_distinct_schedule():
    for name in ["c4", "diamond", "tailed_triangle", "house", "k5e", "k6e",
                 "c6chord03"]:
        a = P.named(name)
        s, c = P.pick_schedule(a, True)
        assert s in P.distinct_schedules(a)
        assert c == min(P.analytic_cost(a, t, True) for t in P.distinct_schedules(a))


# ------------------------------------------------ learned cost model oracle


def test_mlp_oracle_gradient_finite_differences():
    """The oracle's analytic gradient against central finite differences."""
    import numpy as np
    from oracle import mlp
    rng = np.random.Generator(np.random.PCG64(3))
    D, H, n = 7, 5, 11
    P = rng.normal(0, 0.5, H * D + 2 * H + 1)
    X = rng.normal(0, 1, (n, D))
    t = rng.normal(0, 1, n)
    loss, g = mlp.loss_grad(P, X, t, D, H)
    eps = 1e-6
    for i in range(P.size):
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += eps
        Pm[i] -= eps
        fd = (mlp.loss_grad(Pp, X, t, D, H)[0] - mlp.loss_grad(Pm, X, t, D, H)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i
    # forward by hand for one sample
    W1, b1, w2, b2 = mlp.unpack(P, D, H)
    y0 = sum(w2[h] * max(0.0, float(W1[h] @ X[0] + b1[h])) for h in range(H)) + b2
    assert abs(mlp.forward(P, X, D, H)[0][0] - y0) < 1e-12


def test_bf16_rounding_oracle():
    import numpy as np
    from oracle import mlp
    # exactly representable values stay; halfway cases go to even
    assert mlp.bf16(np.array([1.0, -2.5, 0.0]))[0] == 1.0
    one_plus = np.float32(1.0) + np.float32(2 ** -8)   # halfway between 1 and 1+2^-7
    assert mlp.bf16(np.array([one_plus]))[0] == 1.0
    up = np.float32(1.0) + np.float32(3 * 2 ** -9)     # nearer 1+2^-7
    assert mlp.bf16(np.array([up]))[0] == 1.0 + 2 ** -7
