// Internal declarations shared by the host code (graph preparation, pattern
// compiler, C-ABI) and the HIP mining kernels of libgz.
#pragma once

#include <stdint.h>

#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "gz.h"

namespace gz {

constexpr int kMaxK = 8;

// ---------------------------------------------------------------- the plan
//
// Lowered schedule: one descriptor per loop i = 1..k-1 (loop 0 enumerates the
// roots).  Bit j of a mask refers to loop j < i.
//   isect : loops whose vertex is a pattern neighbour of loop i's vertex; the
//           candidates lie in the intersection of their neighbour lists
//   sub   : loops whose vertex is a pattern non-neighbour (vertex-induced mode
//           only); their neighbour lists are subtracted
//   excl  : loops whose graph vertex could equal a candidate and must be
//           excluded explicitly (non-neighbours not already ruled out by the
//           loop's bound chain)
//   bound : the single kept restriction (Theorem 2): candidates must be
//           smaller than the graph vertex of loop `bound`; -1 for none
//   src   : an earlier materialised loop (2 <= src < i) whose candidate set
//           already satisfies a subset of loop i's constraints and whose
//           bound is no tighter; loop i may filter that set instead of
//           intersecting lists; -1 when there is none
//   pos_src / neg_src : isect / sub bits still to check when filtering src
//   acct  : accounting of algorithmic bytes (the instrumented pass only).
//           Bit 7 set when loop i extends the enclosing loop's set: loop
//           i-1 >= 2 is materialised, loop i is bounded by it, and loop
//           i-1's intersected and subtracted lists are subsets of loop i's.
//           Bits 0..6 then name the lists loop i adds; the enclosing set
//           contributes its elements below v_{i-1}.
struct Level {
  uint8_t isect;
  uint8_t sub;
  uint8_t excl;
  int8_t bound;
  int8_t src;
  uint8_t pos_src;
  uint8_t neg_src;
  uint8_t acct;
};

struct Plan {
  int32_t k;
  int32_t induced;
  Level lv[kMaxK];
  int32_t ie_force = 0;  // last loop: inclusion-exclusion for every item (tests)
  // last loop: items whose walk reaches long_min elements are counted by the
  // whole wave, merging probe lists at most merge_ratio / 8 times the walk's
  // length through an LDS window (set per count call)
  int32_t long_min = 1 << 30;
  int32_t merge_ratio = 4;
  // last loop: an item takes inclusion-exclusion when its unit cost (walked
  // elements times probes per element) is below ie_ratio / 8 of the direct
  // evaluation's
  int32_t ie_ratio = 12;
  // last loop: a group of items whose own rows are walked is swept (one LDS
  // mask per block of vertex ids for the earlier loops' lists) when those
  // walks total at least sweep_min entries (0: never); an item keeps
  // inclusion-exclusion when that walks under 1 / sweep_ie of its row
  int32_t sweep_min = 0;
  int32_t sweep_ie = 2;
};

// ---------------------------------------------------------------- patterns

struct Pattern {
  int k = 0;
  uint8_t adj[kMaxK][kMaxK] = {};
};

using Perm = std::vector<int8_t>;  // x[v] = image of label v

std::vector<Perm> automorphisms(const Pattern& p);
bool pattern_connected(const Pattern& p);
bool schedule_valid(const Pattern& p, const int8_t* order);
std::vector<Perm> explore_schedules(const Pattern& p, const std::vector<Perm>& aut);
void reduced_bounds(const Pattern& p, const std::vector<Perm>& aut,
                    const int8_t* order, int8_t* bound);
double analytic_cost(const Pattern& p, const int8_t* order, const int8_t* bound,
                     bool induced);
Plan lower_plan(const Pattern& p, const int8_t* order, const int8_t* bound,
                bool induced);

// ------------------------------------------------------------------ graphs

struct HostGraph {
  int32_t n = 0;
  std::vector<int32_t> rowptr;      // n+1
  std::vector<int32_t> col;         // nnz, ascending rows
  std::vector<int32_t> lo;          // per vertex: neighbours with smaller id
  std::vector<int32_t> old_of_new;  // n
};

// Build a simple symmetric graph from a raw edge list (self-loops and
// duplicates dropped, rows sorted).  Returns false with a message on bad
// input.
bool graph_from_edges(const int32_t* src, const int32_t* dst, int64_t m,
                      int32_t n, HostGraph* out, std::string* err);
// Normalise an arbitrary CSR (same rules as above).
bool graph_from_csr_normalize(const int32_t* rowptr, const int32_t* col,
                              int32_t n, int64_t nnz, HostGraph* out,
                              std::string* err);
// Validate a CSR that must already be simple, symmetric and sorted.
bool graph_from_csr_strict(const int32_t* rowptr, const int32_t* col, int32_t n,
                           int64_t nnz, HostGraph* out, std::string* err);
// Degree reindex: new ids by decreasing degree, ties by increasing old id.
void graph_reindex(HostGraph* g);
// Fill g->lo and the identity mapping where missing.
void graph_finish(HostGraph* g);

void parallel_for(int64_t n, int64_t grain,
                  const std::function<void(int64_t, int64_t)>& body);

// ---------------------------------------------------------------- handles

// Task list of the first loop: root r contributes ceil(len1(r) / chunk)
// tasks, each covering `chunk` consecutive first-loop candidates.
struct DevTasks {
  int64_t* prefix = nullptr;   // device, n_roots + 1 entries
  int64_t n_tasks = 0;
};

// Root lists of the clique path: light roots (3 <= lo <= 64) for the wave
// kernel, heavy roots (64 < lo <= max_lo) for the workgroup kernel, the
// latter in order of decreasing lo so that the largest start first, and the
// roots above max_lo for the generic kernels.  Device arrays.
struct CliqueLists {
  int32_t* light_v = nullptr;
  int32_t* light_r = nullptr;
  int64_t n_light = 0;
  int32_t* heavy_v = nullptr;
  int32_t* heavy_r = nullptr;
  int64_t n_heavy = 0;
  int32_t heavy_max_lo = 0;
  // heavy roots (sorted by candidate count, largest first) fall into
  // contiguous size classes: roots [bucket_begin[b], bucket_begin[b + 1])
  // have rows of at most bucket_w[b] 64-bit words
  int32_t n_buckets = 0;
  int32_t bucket_w[4] = {0, 0, 0, 0};
  int64_t bucket_begin[5] = {0, 0, 0, 0, 0};
  // roots with more candidates than the bit rows hold (max_lo) take the
  // generic loops: vertices, output slots and their first-loop task prefix
  int32_t max_lo = 0;
  int32_t* over_v = nullptr;
  int32_t* over_r = nullptr;
  int64_t* over_prefix = nullptr;
  int64_t n_over = 0;
  int64_t over_tasks = 0;
};

// Dense neighbour bitmaps of the leading vertices 0..n_hub-1, which after
// the degree reindex are the vertices of highest degree: bit x of row v is
// set when x is a neighbour of v.  A membership probe into a hub's list is
// then one load instead of a binary search.  Row v starts at word
// v * row_words (32-bit words, row_words = ceil(n / 32)).
struct HubMaps {
  int32_t min_deg = 0;        // vertices of at least this degree get a row
  long long cap_bytes = 0;    // and at most this many bytes in total
  int32_t n_hub = 0;
  long long row_words = 0;
  uint32_t* bits = nullptr;   // device, n_hub * row_words words
};

void set_error(const std::string& msg);

}  // namespace gz

struct gz_graph {
  gz::HostGraph host;
  int32_t max_deg = 0;
  int32_t max_lo = 0;
  // n, undirected edges, mean degree, E[d^2]/E[d], max degree, mean lo,
  // E[lo^2]/E[lo], max lo (lo: neighbours with a smaller id)
  double stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int device = 0;
  int32_t* d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  int32_t* d_lo = nullptr;
  // first-loop task prefixes over all roots, by (bounded?, chunk) - built on
  // first use and kept for the handle's life
  mutable std::mutex task_mu;
  mutable std::vector<std::pair<int64_t, gz::DevTasks>> task_cache;
  // clique-path root lists over all roots, built on first use
  mutable bool clique_ready = false;
  mutable gz::CliqueLists clique_all;
  // hub bitmaps by (min_deg, cap_bytes), built on first use
  mutable std::vector<gz::HubMaps> hub_cache;
};

struct gz_schedule {
  gz::Pattern pat;
  int induced = 1;
  uint32_t flags = 0;
  int8_t order[gz::kMaxK] = {};
  int8_t bound[gz::kMaxK] = {};
  uint64_t aut_size = 0;
  int32_t n_distinct = 0;
  double cost = 0.0;
  gz::Plan plan{};
};
