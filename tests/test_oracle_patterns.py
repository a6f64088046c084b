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


def test_adam_oracle_first_step_closed_form():
    """From zero moments the bias corrections cancel exactly: the first step
    moves every parameter by -lr g / (|g| + eps).  The tiny gradient pins
    where eps sits (outside the square root: 1e-8 / (1e-8 + 1e-8) = 1/2)."""
    import numpy as np
    from oracle import mlp
    g = np.array([0.5, -2.0, 1e-8, 3.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    z = np.zeros(4)
    p1, m1, v1 = mlp.adam(p0, g, z, z, lr=0.01, step=1)
    assert np.allclose(m1, 0.1 * g, rtol=1e-15, atol=0)
    assert np.allclose(v1, 0.001 * g * g, rtol=1e-15, atol=0)
    assert p1[2] == pytest.approx(3.0 - 0.005, rel=1e-15)
    assert p1[0] == pytest.approx(1.0 - 0.01 * 0.5 / (0.5 + 1e-8), rel=1e-15)
    assert p1[1] == pytest.approx(2.0 + 0.01 * 2.0 / (2.0 + 1e-8), rel=1e-15)
    # a constant gradient keeps the corrected moments at g and g^2: every
    # step is the same
    p, m, v = p0, z, z
    for step in range(1, 6):
        q, m, v = mlp.adam(p, g, m, v, lr=0.01, step=step)
        assert np.allclose(q - p, p1 - p0, rtol=1e-9, atol=0)
        p = q


def test_adam_oracle_second_step_by_hand():
    """Gradients 1 then -2, lr 0.1, beta1 0.9, beta2 0.999, eps 1e-8, from 0:
    m2 = 0.9*0.1 - 0.2 = -0.11, v2 = 0.999*0.001 + 0.004 = 0.004999;
    corrected -0.11/0.19 and 0.004999/0.001999 = 2.5007503751875938;
    p2 = -0.1/(1 + 1e-8) + 0.1 * 0.5789473684210526 / (1.5813761017504956 + 1e-8)
       = -0.06338964652792491 (decimal arithmetic, 40 digits)."""
    import numpy as np
    from oracle import mlp
    z = np.zeros(1)
    p1, m1, v1 = mlp.adam(z, np.array([1.0]), z, z, lr=0.1, step=1)
    assert p1[0] == pytest.approx(-0.09999999900000001, rel=1e-15)
    p2, m2, v2 = mlp.adam(p1, np.array([-2.0]), m1, v1, lr=0.1, step=2)
    assert m2[0] == pytest.approx(-0.11, rel=1e-14)
    assert v2[0] == pytest.approx(0.004999, rel=1e-14)
    assert p2[0] == pytest.approx(-0.06338964652792491, rel=1e-13)


def test_analytic_cost_red_edge_factor_by_hand():
    """Induced path P3 (centre 0, leaves 1 and 2), schedule (0, 1, 2), bound
    v2 < v1: loop 1 has n p iterations per root, loop 2 n p (1-p) (one black,
    one red earlier neighbour), halved by the bound:
    cost = n + n^2 p + n^3 p^2 (1-p) / 2 = 18467.354679441641 at n = 1000,
    p = 5/999; without the red factor (edge-induced) 18530.042555067580."""
    a = P.from_edges(3, [(0, 1), (0, 2)])
    assert P.reduced_bounds(a, (0, 1, 2)) == [-1, -1, 1]
    assert P.analytic_cost(a, (0, 1, 2), True) == pytest.approx(18467.354679441641, rel=1e-13)
    assert P.analytic_cost(a, (0, 1, 2), False) == pytest.approx(18530.042555067580, rel=1e-13)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_analytic_last_loop_is_expected_instances(k):
    """The last loop's iterations in the model are the expected number of
    instances in G(n, p), with n^k in place of n (n-1)...(n-k+1): each of the
    m pattern edges present (p), each of the C(k,2) - m non-edges absent
    (1 - p, vertex-induced only), each instance found once (1/|Aut|).  A red
    factor dropped or counted on the wrong loops changes the exponent of
    (1 - p) and fails here for every non-clique pattern."""
    n, pr = 1000, 5.0 / 999
    for a in P.connected_patterns(k):
        m = sum(a[i][j] for i in range(k) for j in range(i + 1, k))
        aut = len(P.automorphisms(a))
        for s in P.distinct_schedules(a):
            for induced in (True, False):
                red = (k * (k - 1) // 2 - m) if induced else 0
                want = n ** k * pr ** m * (1 - pr) ** red / aut
                got = P.level_iterations(a, s, induced)[-1]
                assert got == pytest.approx(want, rel=1e-12), (a, s, induced)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_explorer_emits_lexicographic_class_minima(k):
    """A second formulation of Algorithm 3's output: group the brute-force
    valid schedules (Algorithm 2) into classes under the automorphisms and
    keep each class's lexicographically smallest member; the explorer emits
    exactly these, in lexicographic order (the order the analytic pick's
    tie-break relies on)."""
    for a in P.connected_patterns(k):
        auts = P.automorphisms(a)
        valid = P.valid_schedules_bruteforce(a)
        minima = sorted({min(tuple(x[v] for v in s) for x in auts) for s in valid})
        assert P.distinct_schedules(a) == minima
