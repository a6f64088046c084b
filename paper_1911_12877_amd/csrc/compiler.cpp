// Pattern compiler (host): automorphism group, schedule explorer, restriction
// generation, analytic cost model and lowering to per-loop descriptors.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "gz_internal.h"

namespace gz {

// Every permutation of the labels that maps edges to edges and non-edges to
// non-edges (Section 4.2: found by trying all k! permutations).
std::vector<Perm> automorphisms(const Pattern& p) {
  std::vector<Perm> out;
  Perm x(p.k);
  std::iota(x.begin(), x.end(), 0);
  do {
    bool ok = true;
    for (int a = 0; a < p.k && ok; ++a)
      for (int b = a + 1; b < p.k && ok; ++b)
        ok = p.adj[x[a]][x[b]] == p.adj[a][b];
    if (ok) out.push_back(x);
  } while (std::next_permutation(x.begin(), x.end()));
  return out;
}

static uint32_t nbr_mask(const Pattern& p, int v) {
  uint32_t m = 0;
  for (int u = 0; u < p.k; ++u)
    if (p.adj[v][u]) m |= 1u << u;
  return m;
}

bool pattern_connected(const Pattern& p) {
  if (p.k <= 0) return false;
  uint32_t seen = 1, frontier = 1;
  while (frontier) {
    uint32_t next = 0;
    for (int v = 0; v < p.k; ++v)
      if (frontier >> v & 1) next |= nbr_mask(p, v);
    frontier = next & ~seen;
    seen |= next;
  }
  return seen == (1u << p.k) - 1;
}

bool schedule_valid(const Pattern& p, const int8_t* order) {
  uint32_t used = 0;
  for (int i = 0; i < p.k; ++i) {
    int v = order[i];
    if (v < 0 || v >= p.k || (used >> v & 1)) return false;
    if (i > 0 && !(nbr_mask(p, v) & used)) return false;
    used |= 1u << v;
  }
  return true;
}

// Orbits of a permutation group on a set of labels: orbit_of[v] is the
// smallest label of v's orbit (for v in `set`; the set must be closed under
// the group).
static void orbit_minima(const std::vector<Perm>& group, uint32_t set, int k, int8_t* orbit_of) {
  for (int v = 0; v < k; ++v) orbit_of[v] = (int8_t)v;
  for (int v = 0; v < k; ++v) {
    if (!(set >> v & 1)) continue;
    for (const Perm& g : group) orbit_of[v] = std::min<int8_t>(orbit_of[v], g[v]);
  }
}

// The pointwise stabiliser of v within a group.
static std::vector<Perm> fixing(const std::vector<Perm>& group, int v) {
  std::vector<Perm> out;
  for (const Perm& g : group)
    if (g[v] == v) out.push_back(g);
  return out;
}

// Distinct schedules (Algorithm 3).  Two prefixes that an automorphism maps
// onto each other have the same completions up to that automorphism, so of
// the vertices that may come next (all of them first, afterwards the
// unscheduled neighbours of the prefix) only one per orbit of the group
// fixing the prefix pointwise is tried: the orbit's smallest label, in
// ascending order.  `group` fixes the prefix; `frontier` holds the
// unscheduled neighbours of the prefix.
static void distinct_orders(const Pattern& p, Perm& prefix, uint32_t placed,
                            const std::vector<Perm>& group, uint32_t frontier,
                            std::vector<Perm>* out) {
  if ((int)prefix.size() == p.k) {
    out->push_back(prefix);
    return;
  }
  const uint32_t next = prefix.empty() ? (1u << p.k) - 1 : frontier;
  int8_t orbit_of[kMaxK];
  orbit_minima(group, next, p.k, orbit_of);
  for (int v = 0; v < p.k; ++v) {
    if (!(next >> v & 1) || orbit_of[v] != v) continue;  // one per orbit
    prefix.push_back((int8_t)v);
    const uint32_t now = placed | (1u << v);
    distinct_orders(p, prefix, now, fixing(group, v), (frontier | nbr_mask(p, v)) & ~now, out);
    prefix.pop_back();
  }
}

std::vector<Perm> explore_schedules(const Pattern& p, const std::vector<Perm>& aut) {
  std::vector<Perm> out;
  Perm prefix;
  distinct_orders(p, prefix, 0u, aut, 0u, &out);
  return out;
}

// Restrictions (Algorithm 1) reduced to one bound per loop (Theorem 2), from
// the stabiliser chain of the schedule: G_0 = Aut and G_{i+1} = the elements
// of G_i fixing the i-th scheduled vertex v_i.  Every other member u of v_i's
// orbit under G_i must get a smaller id than v_i; of all such relations on u
// the one with the latest v_i is kept (it implies the earlier ones), so
// bound(u) = the position of the last v_i whose G_i-orbit contains u.
void reduced_bounds(const Pattern& p, const std::vector<Perm>& aut,
                    const int8_t* order, int8_t* bound) {
  int last[kMaxK];  // position of the last scheduled vertex bounding u
  for (int u = 0; u < p.k; ++u) last[u] = -1;
  std::vector<Perm> chain = aut;
  for (int i = 0; i < p.k; ++i) {
    const int v = order[i];
    uint32_t orbit = 0;
    for (const Perm& g : chain) orbit |= 1u << g[v];
    for (int u = 0; u < p.k; ++u)
      if (u != v && (orbit >> u & 1)) last[u] = i;
    chain = fixing(chain, v);
  }
  for (int i = 0; i < p.k; ++i) bound[i] = (int8_t)last[order[i]];
}

// Section 5.4 and the appendix.  In G(n, p) with n = 1000 and average degree
// 5, a loop whose candidates come from c earlier pattern neighbours and d
// earlier non-neighbours (d counted only when vertex-induced) runs
// n p^c (1-p)^d times per enclosing iteration.  The fraction of iterations
// up to loop i that pass every restriction is the product over loops j <= i
// of 1/z_j, z_j = size of j's subtree in the forest of kept bounds among
// loops 0..i.  The cost is the sum over loops of (product of loop sizes) x
// (pass fraction).
double analytic_cost(const Pattern& p, const int8_t* order, const int8_t* bound,
                     bool induced) {
  const double n = 1000.0, pr = 5.0 / 999.0;
  double total = 0.0, prod = 1.0;
  for (int i = 0; i < p.k; ++i) {
    double size;
    if (i == 0) {
      size = n;
    } else {
      int c = 0;
      for (int j = 0; j < i; ++j) c += p.adj[order[j]][order[i]] ? 1 : 0;
      int d = induced ? (i - c) : 0;
      size = n * std::pow(pr, c) * std::pow(1.0 - pr, d);
    }
    prod *= size;
    int z[kMaxK];
    for (int j = 0; j <= i; ++j) z[j] = 1;
    for (int j = i; j >= 1; --j)
      if (bound[j] >= 0) z[bound[j]] += z[j];
    double rate = 1.0;
    for (int j = 0; j <= i; ++j) rate /= z[j];
    total += prod * rate;
  }
  return total;
}

// true when loop a is b or lies on b's chain of bounds (so v_b <= v_a)
static bool on_bound_chain(const int8_t* bound, int b, int a) {
  for (int x = b; x >= 0; x = bound[x])
    if (x == a) return true;
  return false;
}

Plan lower_plan(const Pattern& p, const int8_t* order, const int8_t* bound,
                bool induced) {
  Plan plan{};
  plan.k = p.k;
  plan.induced = induced ? 1 : 0;
  for (int i = 0; i < kMaxK; ++i) plan.lv[i] = Level{0, 0, 0, -1, -1, 0, 0, 0};
  for (int i = 1; i < p.k; ++i) {
    Level& L = plan.lv[i];
    for (int j = 0; j < i; ++j) {
      if (p.adj[order[j]][order[i]])
        L.isect |= (uint8_t)(1u << j);
      else if (induced)
        L.sub |= (uint8_t)(1u << j);
    }
    L.bound = bound[i];
    for (int j = 0; j < i; ++j) {
      bool adjacent = L.isect >> j & 1;
      bool implied = L.bound >= 0 && on_bound_chain(bound, L.bound, j);
      if (!adjacent && !implied) L.excl |= (uint8_t)(1u << j);
    }
  }
  // byte accounting: extension of the enclosing loop's set
  for (int i = 3; i < p.k; ++i) {
    Level& L = plan.lv[i];
    const Level& E = plan.lv[i - 1];
    if (L.bound == i - 1 && !(E.isect & ~L.isect) && !(E.sub & ~L.sub))
      L.acct = (uint8_t)(0x80u | ((L.isect | L.sub) & ~(E.isect | E.sub)));
  }
  // reusable materialised sets: loops 2..k-2 are materialised
  for (int i = 3; i < p.k; ++i) {
    Level& L = plan.lv[i];
    int best = -1, best_w = -1;
    for (int s = 2; s < i && s <= p.k - 2; ++s) {
      const Level& S = plan.lv[s];
      if ((S.isect & ~L.isect) || (S.sub & ~L.sub)) continue;
      bool ok = S.bound < 0 || (L.bound >= 0 && on_bound_chain(bound, L.bound, S.bound));
      if (!ok) continue;
      int w = __builtin_popcount(S.isect) + __builtin_popcount(S.sub);
      if (w >= best_w) {
        best = s;
        best_w = w;
      }
    }
    L.src = (int8_t)best;
    if (best >= 0) {
      L.pos_src = (uint8_t)(L.isect & ~plan.lv[best].isect);
      L.neg_src = (uint8_t)(L.sub & ~plan.lv[best].sub);
    }
  }
  return plan;
}

}  // namespace gz
