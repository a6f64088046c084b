"""Oracle, pattern side: plain Python restatements of the paper's compile-time
algorithms.  TEST INFRASTRUCTURE ONLY: nothing on the product path imports
this module; only tests, the smoke check and the benchmark's CPU-baseline leg
use it.

A pattern is a k x k 0/1 adjacency matrix (list of lists or numpy array),
symmetric with a zero diagonal.  Pattern vertices are labelled 0..k-1.
A schedule is a tuple of the k labels in discovery order (Section 2.1: a total
order on the labels).  A permutation ``x`` is a tuple with ``x[v]`` the image
of label ``v``.

Readings of the paper taken here (each also listed in the design notes):
* Restriction direction: a relation (S[i], S[j]) means the graph vertex mapped
  to S[i] has the LARGER id (Theorem 1).
* Algorithm 3 is called with the full automorphism group and an empty
  candidate set; the next candidate set is (valid_next U N(v)) minus the
  scheduled vertices and v; the "processed" marks belong to one call frame;
  candidates are visited in ascending label order.
* Performance model: uniform random graph with n = 1000 and average degree 5,
  p = 5 / (n - 1).  A loop whose candidates come from c earlier black
  neighbours and d earlier red ones (d = 0 when not vertex-induced) has
  n * p**c * (1-p)**d iterations per enclosing iteration; the restriction
  pass rate up to loop i is the product of 1/z over the forest of the kept
  restrictions among loops 0..i (Appendix, performance model); the cost is
  the sum over loops of (product of loop sizes) * (pass rate).
"""

from __future__ import annotations

import itertools
import math

# ----------------------------------------------------------------- basics


def as_adj(adj):
    k = len(adj)
    a = [[int(adj[i][j]) for j in range(k)] for i in range(k)]
    for i in range(k):
        if a[i][i]:
            raise ValueError("pattern has a self-loop")
        for j in range(k):
            if a[i][j] != a[j][i]:
                raise ValueError("pattern is not symmetric")
    return a


def from_edges(k, edges):
    a = [[0] * k for _ in range(k)]
    for u, v in edges:
        a[u][v] = a[v][u] = 1
    return a


def neighbours(adj, v):
    return [u for u in range(len(adj)) if adj[v][u]]


def is_connected(adj):
    k = len(adj)
    if k == 0:
        return False
    seen = {0}
    stack = [0]
    while stack:
        v = stack.pop()
        for u in neighbours(adj, v):
            if u not in seen:
                seen.add(u)
                stack.append(u)
    return len(seen) == k


# ------------------------------------------------- automorphisms (Sec. 4.2)


def automorphisms(adj):
    """All permutations of the labels that preserve the pattern, found by
    trying every permutation (Section 4.2, first step of Algorithm 1)."""
    adj = as_adj(adj)
    k = len(adj)
    out = []
    for x in itertools.permutations(range(k)):
        if all(adj[x[a]][x[b]] == adj[a][b] for a in range(k) for b in range(k)):
            out.append(x)
    return out


# ------------------------------------------- restrictions (Alg. 1, Thm. 2)


def restrictions(adj, schedule):
    """Algorithm 1: walk the schedule; every automorphism of the current
    group that moves v adds the relation (v, x(v)); the group then shrinks to
    the automorphisms that fix v.  Returns the list of label pairs (a, b),
    meaning id(M(a)) > id(M(b)), in the order they were added."""
    group = automorphisms(adj)
    rel = []
    for v in schedule:
        stabiliser = []
        for x in group:
            if x[v] == v:
                stabiliser.append(x)
            elif (v, x[v]) not in rel:
                rel.append((v, x[v]))
        group = stabiliser
    return rel


def reduced_bounds(adj, schedule):
    """Theorem 2: for every schedule position k keep only the relation
    (S[z], S[k]) with the largest z.  Returns bound[k] = z (a schedule
    position) or -1 when position k has no upper bound."""
    pos = {v: i for i, v in enumerate(schedule)}
    k = len(schedule)
    bound = [-1] * k
    for a, b in restrictions(adj, schedule):
        z, t = pos[a], pos[b]
        if z > bound[t]:
            bound[t] = z
    return bound


def relations_as_positions(adj, schedule):
    pos = {v: i for i, v in enumerate(schedule)}
    return [(pos[a], pos[b]) for a, b in restrictions(adj, schedule)]


# ---------------------------------------- schedules (Alg. 2, Alg. 3, Thm. 3)


def is_valid_schedule(adj, schedule):
    """Section 5.2: every vertex after the first has a black edge to an
    earlier one."""
    for i in range(1, len(schedule)):
        if not any(adj[schedule[j]][schedule[i]] for j in range(i)):
            return False
    return True


def valid_schedules_bruteforce(adj):
    """Algorithm 2: all permutations, keep the valid ones."""
    adj = as_adj(adj)
    return [s for s in itertools.permutations(range(len(adj)))
            if is_valid_schedule(adj, s)]


def valid_schedules_recursive(adj):
    """The recursive smart brute force of Section 5.2: extend a partial
    schedule only by vertices adjacent to it."""
    adj = as_adj(adj)
    k = len(adj)
    out = []

    def rec(sched):
        if len(sched) == k:
            out.append(tuple(sched))
            return
        if not sched:
            nxt = list(range(k))
        else:
            nxt = [u for u in range(k) if u not in sched
                   and any(adj[u][w] for w in sched)]
        for v in nxt:
            rec(sched + [v])

    rec([])
    return out


def distinct_schedules(adj):
    """Algorithm 3: the schedule explorer.  At each step the candidates are
    split into orbits of the automorphisms that fix the scheduled vertices;
    only the first member of each orbit is expanded."""
    adj = as_adj(adj)
    k = len(adj)
    out = []

    def rec(sched, group, valid_next):
        if len(sched) == k:
            out.append(tuple(sched))
            return
        iterate_over = list(range(k)) if not sched else sorted(valid_next)
        processed = set()
        for v in iterate_over:
            if v in processed:
                continue
            stabiliser = []
            for x in group:
                if x[v] == v:
                    stabiliser.append(x)
                else:
                    processed.add(x[v])
            nxt = (set(valid_next) | set(neighbours(adj, v))) - set(sched) - {v}
            rec(sched + [v], stabiliser, nxt)

    rec([], automorphisms(adj), set())
    return out


# ------------------------------------ performance model (Sec. 5.4, appendix)


def forest_pass_rate(bound, upto):
    """Probability that independent uniform values x_0..x_upto satisfy
    x_j < x_bound[j] for every j <= upto with a bound: the product over those
    levels of 1/z_j, z_j = 1 + number of levels <= upto below j in the
    restriction forest (appendix, performance model)."""
    z = [1] * (upto + 1)
    for j in range(upto, 0, -1):        # children have larger positions
        p = bound[j]
        if p >= 0:
            z[p] += z[j]
    r = 1.0
    for j in range(upto + 1):
        r /= z[j]
    return r


def level_iterations(adj, schedule, induced, n=1000, avg_deg=5.0):
    """Section 5.4: expected iterations of each loop i in G(n, p), i.e. the
    product of the loop sizes up to i times the restriction pass rate up to
    i.  Returned per loop, in schedule order."""
    adj = as_adj(adj)
    k = len(schedule)
    p = avg_deg / (n - 1)
    bound = reduced_bounds(adj, schedule)
    out = []
    prod = 1.0
    for i in range(k):
        if i == 0:
            size = float(n)
        else:
            c = sum(1 for j in range(i) if adj[schedule[j]][schedule[i]])
            d = (i - c) if induced else 0
            size = n * (p ** c) * ((1.0 - p) ** d)
        prod *= size
        out.append(prod * forest_pass_rate(bound, i))
    return out


def analytic_cost(adj, schedule, induced, n=1000, avg_deg=5.0):
    """Section 5.4: expected loop iterations in G(n, p) summed over loops."""
    total = 0.0
    for it in level_iterations(adj, schedule, induced, n, avg_deg):
        total += it
    return total


def pick_schedule(adj, induced, n=1000, avg_deg=5.0, rel_tol=1e-12):
    """The lowest-cost distinct schedule; costs within ``rel_tol`` of the
    best count as ties, and ties go to the schedule Algorithm 3 emitted
    first."""
    best = None
    best_cost = None
    for s in distinct_schedules(adj):
        c = analytic_cost(adj, s, induced, n, avg_deg)
        if best is None or c < best_cost * (1.0 - rel_tol):
            best, best_cost = s, c
    return best, best_cost


# --------------------------------------------- pattern enumeration (motifs)


def _code(adj, perm):
    k = len(adj)
    c = 0
    for i in range(k):
        for j in range(i + 1, k):
            c = (c << 1) | adj[perm[i]][perm[j]]
    return c


def canonical_code(adj):
    """Largest upper-triangle bit string over all relabellings."""
    k = len(adj)
    return max(_code(adj, p) for p in itertools.permutations(range(k)))


def connected_patterns(k):
    """All connected k-vertex graphs up to isomorphism, as adjacency
    matrices, ordered by (edge count, canonical code)."""
    pairs = [(i, j) for i in range(k) for j in range(i + 1, k)]
    seen = {}
    for mask in range(1 << len(pairs)):
        adj = [[0] * k for _ in range(k)]
        for b, (i, j) in enumerate(pairs):
            if mask >> b & 1:
                adj[i][j] = adj[j][i] = 1
        if not is_connected(adj):
            continue
        code = canonical_code(adj)
        if code not in seen:
            seen[code] = adj
    items = sorted(seen.items(), key=lambda kv: (bin(kv[0]).count("1"), kv[0]))
    return [a for _, a in items]


# ----------------------------------------------------------- named patterns


def named(name):
    """A few patterns by name.  'house' is a 4-cycle 0-1-2-3 with a roof
    vertex 4 joined to 0 and 1; 'c6chord03' / 'c6chord02' are the 6-cycle with
    the chord {0,3} / {0,2}; 'k{n}e' is K_n minus the edge {n-2, n-1}."""
    if name == "triangle":
        return from_edges(3, [(0, 1), (1, 2), (0, 2)])
    if name.startswith("k") and name[1:].isdigit():
        n = int(name[1:])
        return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    if name.startswith("k") and name.endswith("e") and name[1:-1].isdigit():
        n = int(name[1:-1])
        return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)
                              if (i, j) != (n - 2, n - 1)])
    if name.startswith("c") and name[1:].isdigit():
        n = int(name[1:])
        return from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    if name.startswith("p") and name[1:].isdigit():
        n = int(name[1:])
        return from_edges(n, [(i, i + 1) for i in range(n - 1)])
    if name.startswith("star") and name[4:].isdigit():
        n = int(name[4:])
        return from_edges(n, [(0, i) for i in range(1, n)])
    if name == "diamond":
        return from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)])
    if name == "tailed_triangle":
        return from_edges(4, [(0, 1), (1, 2), (0, 2), (0, 3)])
    if name == "house":
        return from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4)])
    if name == "c6chord03":
        return from_edges(6, [(i, (i + 1) % 6) for i in range(6)] + [(0, 3)])
    if name == "c6chord02":
        return from_edges(6, [(i, (i + 1) % 6) for i in range(6)] + [(0, 2)])
    raise KeyError(name)


def multiplicity(adj):
    return len(automorphisms(adj))


def restricted_pass_product(adj, schedule):
    """Product of z over the full schedule (equals |Aut| by the appendix's
    closing remark); returned as an integer."""
    bound = reduced_bounds(adj, schedule)
    return round(1.0 / forest_pass_rate(bound, len(schedule) - 1))


def choose2(x):
    return x * (x - 1) // 2


def falling(n, k):
    return math.perm(n, k)
