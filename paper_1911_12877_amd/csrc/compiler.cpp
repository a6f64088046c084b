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

// Algorithm 3.  Candidates of the next step are visited in ascending label
// order; the automorphisms that fix the scheduled prefix split them into
// orbits and only the first member of each orbit is expanded.  The candidate
// set of the child is (valid_next U N(v)) without the scheduled vertices.
static void explore_rec(const Pattern& p, Perm& sched, uint32_t in_sched,
                        const std::vector<Perm>& group, uint32_t valid_next,
                        std::vector<Perm>* out) {
  if ((int)sched.size() == p.k) {
    out->push_back(sched);
    return;
  }
  uint32_t iterate = sched.empty() ? (1u << p.k) - 1 : valid_next;
  uint32_t processed = 0;
  for (int v = 0; v < p.k; ++v) {
    if (!(iterate >> v & 1) || (processed >> v & 1)) continue;
    std::vector<Perm> stab;
    for (const Perm& x : group) {
      if (x[v] == v)
        stab.push_back(x);
      else
        processed |= 1u << x[v];
    }
    sched.push_back((int8_t)v);
    uint32_t now = in_sched | (1u << v);
    explore_rec(p, sched, now, stab, (valid_next | nbr_mask(p, v)) & ~now, out);
    sched.pop_back();
  }
}

std::vector<Perm> explore_schedules(const Pattern& p, const std::vector<Perm>& aut) {
  std::vector<Perm> out;
  Perm sched;
  explore_rec(p, sched, 0u, aut, 0u, &out);
  return out;
}

// Algorithm 1 in the map form of Section 4.3: walking the schedule, every
// automorphism x of the current group that moves v records "x(v) is bounded
// by v"; a later v overwrites, which keeps the latest position (Theorem 2).
// The group then shrinks to the automorphisms fixing v.
void reduced_bounds(const Pattern& p, const std::vector<Perm>& aut,
                    const int8_t* order, int8_t* bound) {
  int pos[kMaxK];
  for (int i = 0; i < p.k; ++i) pos[order[i]] = i;
  int by[kMaxK];
  for (int v = 0; v < p.k; ++v) by[v] = -1;
  std::vector<Perm> group = aut;
  for (int i = 0; i < p.k; ++i) {
    int v = order[i];
    std::vector<Perm> keep;
    for (const Perm& x : group) {
      if (x[v] == v)
        keep.push_back(x);
      else
        by[x[v]] = v;
    }
    group.swap(keep);
  }
  for (int i = 0; i < p.k; ++i) bound[i] = (int8_t)(by[order[i]] < 0 ? -1 : pos[by[order[i]]]);
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
