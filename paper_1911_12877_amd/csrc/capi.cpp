// C-ABI entry points of libgz (declared in include/gz.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

#include "gz_internal.h"

namespace gz {

gz_status run_count(const gz_graph* g, const gz_schedule* s, hipStream_t st,
                    const int32_t* roots, int64_t n_roots, uint64_t* per_root,
                    bool instr, unsigned __int128* total, unsigned __int128* bytes,
                    float* kernel_ms, bool clique_ops = false);
void free_graph_tasks(gz_graph* g);
gz_status prepare_graph_tasks(const gz_graph* g, hipStream_t st);
gz_status run_count_noalloc(const gz_graph* g, const gz_schedule* s, hipStream_t st,
                            unsigned __int128* total);
gz_status device_prepare_edges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                               bool device_inputs, bool reindex, hipStream_t st, gz_graph* g);

gz_status census_create(const gz_graph* const* graphs, int32_t n_graphs,
                        const gz_schedule* const* scheds, int32_t n_scheds, void** out);
gz_status census_run(void* c, uint64_t* counts, float* ms);
gz_status census_tune(void* c, int32_t* params, float* best_ms);
void census_free(void* c);

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace gz

using namespace gz;

namespace {

#define GZ_CHECK_HIP(call)                                                \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return GZ_EDEVICE;                                                  \
    }                                                                     \
  } while (0)

gz_status upload_graph(gz_graph* g, hipStream_t st) {
  const HostGraph& h = g->host;
  GZ_CHECK_HIP(hipGetDevice(&g->device));
  const size_t nnz = h.col.size();
  GZ_CHECK_HIP(hipMalloc(&g->d_rowptr, sizeof(int32_t) * (h.n + 1)));
  GZ_CHECK_HIP(hipMalloc(&g->d_col, sizeof(int32_t) * std::max<size_t>(nnz, 1)));
  GZ_CHECK_HIP(hipMalloc(&g->d_lo, sizeof(int32_t) * std::max<int32_t>(h.n, 1)));
  GZ_CHECK_HIP(hipMemcpyAsync(g->d_rowptr, h.rowptr.data(), sizeof(int32_t) * (h.n + 1),
                              hipMemcpyHostToDevice, st));
  if (nnz)
    GZ_CHECK_HIP(hipMemcpyAsync(g->d_col, h.col.data(), sizeof(int32_t) * nnz,
                                hipMemcpyHostToDevice, st));
  if (h.n)
    GZ_CHECK_HIP(hipMemcpyAsync(g->d_lo, h.lo.data(), sizeof(int32_t) * h.n,
                                hipMemcpyHostToDevice, st));
  GZ_CHECK_HIP(hipStreamSynchronize(st));
  return GZ_OK;
}

void release_graph(gz_graph* g) {
  if (!g) return;
  free_graph_tasks(g);
  if (g->d_rowptr) (void)hipFree(g->d_rowptr);
  if (g->d_col) (void)hipFree(g->d_col);
  if (g->d_lo) (void)hipFree(g->d_lo);
  delete g;
}

// Copy device input arrays to host when the caller passed device pointers.
gz_status host_copy(const int32_t* p, size_t count, bool device, hipStream_t st,
                    std::vector<int32_t>* keep, const int32_t** out) {
  if (!device || count == 0) {
    *out = p;
    return GZ_OK;
  }
  keep->resize(count);
  GZ_CHECK_HIP(hipMemcpyAsync(keep->data(), p, sizeof(int32_t) * count,
                              hipMemcpyDeviceToHost, st));
  GZ_CHECK_HIP(hipStreamSynchronize(st));
  *out = keep->data();
  return GZ_OK;
}

// Degree statistics of a prepared graph (cost-model features).
void graph_stats(gz_graph* g) {
  const HostGraph& h = g->host;
  double sd = 0, sd2 = 0, sl = 0, sl2 = 0;
  for (int32_t v = 0; v < h.n; ++v) {
    const double d = h.rowptr[v + 1] - h.rowptr[v], l = h.lo[v];
    g->max_deg = std::max(g->max_deg, h.rowptr[v + 1] - h.rowptr[v]);
    g->max_lo = std::max(g->max_lo, h.lo[v]);
    sd += d;
    sd2 += d * d;
    sl += l;
    sl2 += l * l;
  }
  const double n = std::max<double>(h.n, 1);
  g->stats[0] = h.n;
  g->stats[1] = sd / 2;
  g->stats[2] = sd / n;
  g->stats[3] = sd > 0 ? sd2 / sd : 0;
  g->stats[4] = g->max_deg;
  g->stats[5] = sl / n;
  g->stats[6] = sl > 0 ? sl2 / sl : 0;
  g->stats[7] = g->max_lo;
}

gz_status finish_graph(gz_graph* g, uint32_t flags, hipStream_t st, gz_graph** out) {
  if (!(flags & GZ_GRAPH_NO_REINDEX)) graph_reindex(&g->host);
  graph_finish(&g->host);
  graph_stats(g);
  gz_status rc = upload_graph(g, st);
  if (!rc) rc = prepare_graph_tasks(g, st);
  if (rc) {
    release_graph(g);
    return rc;
  }
  *out = g;
  return GZ_OK;
}

bool read_pattern(const uint8_t* adj, int32_t k, Pattern* p) {
  if (!adj) {
    set_error("pattern adjacency is NULL");
    return false;
  }
  if (k < 2 || k > kMaxK) {
    set_error("pattern size must be between 2 and 8");
    return false;
  }
  p->k = k;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      uint8_t a = adj[i * k + j];
      if (a > 1) {
        set_error("pattern adjacency entries must be 0 or 1");
        return false;
      }
      p->adj[i][j] = a;
    }
  for (int i = 0; i < k; ++i) {
    if (p->adj[i][i]) {
      set_error("pattern has a self-loop");
      return false;
    }
    for (int j = 0; j < k; ++j)
      if (p->adj[i][j] != p->adj[j][i]) {
        set_error("pattern adjacency is not symmetric");
        return false;
      }
  }
  if (!pattern_connected(*p)) {
    set_error("pattern is not connected");
    return false;
  }
  return true;
}

gz_status build_schedule(const Pattern& p, int32_t induced, uint32_t flags,
                         const int8_t* order, gz_schedule** out) {
  if (!out) {
    set_error("output handle pointer is NULL");
    return GZ_EINVAL;
  }
  if (flags & ~(uint32_t)GZ_SCHED_NO_RESTRICT) {
    set_error("unknown schedule flags");
    return GZ_EINVAL;
  }
  std::vector<Perm> aut = automorphisms(p);
  std::vector<Perm> ds = explore_schedules(p, aut);
  auto* s = new (std::nothrow) gz_schedule();
  if (!s) {
    set_error("out of host memory");
    return GZ_ENOMEM;
  }
  s->pat = p;
  s->induced = induced ? 1 : 0;
  s->flags = flags;
  s->aut_size = aut.size();
  s->n_distinct = (int32_t)ds.size();
  if (order) {
    std::copy(order, order + p.k, s->order);
    reduced_bounds(p, aut, s->order, s->bound);
    s->cost = analytic_cost(p, s->order, s->bound, induced != 0);
  } else {
    // cheapest distinct schedule; costs within a relative 1e-12 of the best
    // are ties, won by the schedule the explorer emitted first
    bool have = false;
    for (const Perm& x : ds) {
      int8_t b[kMaxK];
      reduced_bounds(p, aut, x.data(), b);
      double c = analytic_cost(p, x.data(), b, induced != 0);
      if (!have || c < s->cost * (1.0 - 1e-12)) {
        have = true;
        s->cost = c;
        std::copy(x.begin(), x.end(), s->order);
        std::copy(b, b + p.k, s->bound);
      }
    }
  }
  int8_t kb[kMaxK];
  for (int i = 0; i < p.k; ++i) kb[i] = (flags & GZ_SCHED_NO_RESTRICT) ? -1 : s->bound[i];
  s->plan = lower_plan(p, s->order, kb, induced != 0);
  *out = s;
  return GZ_OK;
}

}  // namespace

namespace gz {
bool read_pattern_checked(const uint8_t* adj, int32_t k, Pattern* p) { return read_pattern(adj, k, p); }
gz_status build_schedule_for(const Pattern& p, int32_t induced, uint32_t flags, const int8_t* order,
                             gz_schedule** out) {
  return build_schedule(p, induced, flags, order, out);
}
}  // namespace gz

extern "C" {

gz_status gz_load_graph(const int32_t* rowptr, const int32_t* colidx, int32_t n,
                        int64_t nnz, uint32_t flags, void* hip_stream, gz_graph** out) {
  if (!out || !rowptr || (nnz > 0 && !colidx)) {
    set_error("NULL argument");
    return GZ_EINVAL;
  }
  if (flags & ~(uint32_t)(GZ_GRAPH_NORMALIZE | GZ_GRAPH_NO_REINDEX | GZ_GRAPH_DEVICE_PTRS)) {
    set_error("unknown graph flags");
    return GZ_EINVAL;
  }
  if (n < 0 || nnz < 0 || nnz > INT32_MAX) {
    set_error("n or nnz out of range");
    return GZ_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const bool dev = flags & GZ_GRAPH_DEVICE_PTRS;
  std::vector<int32_t> hr, hc;
  const int32_t *r = nullptr, *c = nullptr;
  gz_status rc = host_copy(rowptr, (size_t)n + 1, dev, st, &hr, &r);
  if (!rc) rc = host_copy(colidx, (size_t)nnz, dev, st, &hc, &c);
  if (rc) return rc;
  auto* g = new (std::nothrow) gz_graph();
  if (!g) {
    set_error("out of host memory");
    return GZ_ENOMEM;
  }
  std::string err;
  bool ok = (flags & GZ_GRAPH_NORMALIZE)
                ? graph_from_csr_normalize(r, c, n, nnz, &g->host, &err)
                : graph_from_csr_strict(r, c, n, nnz, &g->host, &err);
  if (!ok) {
    delete g;
    set_error(err);
    return GZ_EINVAL;
  }
  return finish_graph(g, flags, st, out);
}

gz_status gz_load_edges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                        uint32_t flags, void* hip_stream, gz_graph** out) {
  if (!out || (m > 0 && (!src || !dst))) {
    set_error("NULL argument");
    return GZ_EINVAL;
  }
  if (flags & ~(uint32_t)(GZ_GRAPH_NORMALIZE | GZ_GRAPH_NO_REINDEX | GZ_GRAPH_DEVICE_PTRS |
                          GZ_GRAPH_PREP_DEVICE)) {
    set_error("unknown graph flags");
    return GZ_EINVAL;
  }
  if (n < 0 || m < 0) {
    set_error("n or m out of range");
    return GZ_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const bool dev = flags & GZ_GRAPH_DEVICE_PTRS;
  if (flags & GZ_GRAPH_PREP_DEVICE) {
    auto* g = new (std::nothrow) gz_graph();
    if (!g) {
      set_error("out of host memory");
      return GZ_ENOMEM;
    }
    gz_status rc = device_prepare_edges(src, dst, m, n, dev, !(flags & GZ_GRAPH_NO_REINDEX), st, g);
    if (!rc) {
      graph_stats(g);
      rc = prepare_graph_tasks(g, st);
    }
    if (rc) {
      release_graph(g);
      return rc;
    }
    *out = g;
    return GZ_OK;
  }
  std::vector<int32_t> hs, hd;
  const int32_t *s = nullptr, *d = nullptr;
  gz_status rc = host_copy(src, (size_t)m, dev, st, &hs, &s);
  if (!rc) rc = host_copy(dst, (size_t)m, dev, st, &hd, &d);
  if (rc) return rc;
  auto* g = new (std::nothrow) gz_graph();
  if (!g) {
    set_error("out of host memory");
    return GZ_ENOMEM;
  }
  std::string err;
  if (!graph_from_edges(s, d, m, n, &g->host, &err)) {
    delete g;
    set_error(err);
    return GZ_EINVAL;
  }
  return finish_graph(g, flags, st, out);
}

gz_status gz_graph_info(const gz_graph* g, int32_t* n, int64_t* nnz, int32_t* max_deg,
                        int32_t* max_lo_deg) {
  if (!g) {
    set_error("NULL graph");
    return GZ_EINVAL;
  }
  if (n) *n = g->host.n;
  if (nnz) *nnz = (int64_t)g->host.col.size();
  if (max_deg) *max_deg = g->max_deg;
  if (max_lo_deg) *max_lo_deg = g->max_lo;
  return GZ_OK;
}

gz_status gz_graph_export(const gz_graph* g, int32_t* rowptr, int32_t* colidx,
                          int32_t* old_of_new) {
  if (!g) {
    set_error("NULL graph");
    return GZ_EINVAL;
  }
  const HostGraph& h = g->host;
  if (rowptr) std::copy(h.rowptr.begin(), h.rowptr.end(), rowptr);
  if (colidx) std::copy(h.col.begin(), h.col.end(), colidx);
  if (old_of_new) std::copy(h.old_of_new.begin(), h.old_of_new.end(), old_of_new);
  return GZ_OK;
}

void gz_free_graph(gz_graph* g) { release_graph(g); }

gz_status gz_prepare_edges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                           uint32_t flags, int64_t* nnz_out, int32_t* rowptr_out,
                           int32_t* colidx_out, int32_t* old_of_new_out, int32_t* lo_out) {
  if ((m > 0 && (!src || !dst || !colidx_out)) || !rowptr_out || !nnz_out) {
    set_error("NULL argument");
    return GZ_EINVAL;
  }
  if (flags & ~(uint32_t)(GZ_GRAPH_NORMALIZE | GZ_GRAPH_NO_REINDEX)) {
    set_error("unknown or unsupported flags for host preparation");
    return GZ_EINVAL;
  }
  HostGraph h;
  std::string err;
  if (!graph_from_edges(src, dst, m, n, &h, &err)) {
    set_error(err);
    return GZ_EINVAL;
  }
  if (!(flags & GZ_GRAPH_NO_REINDEX)) graph_reindex(&h);
  graph_finish(&h);
  *nnz_out = (int64_t)h.col.size();
  std::copy(h.rowptr.begin(), h.rowptr.end(), rowptr_out);
  std::copy(h.col.begin(), h.col.end(), colidx_out);
  if (old_of_new_out) std::copy(h.old_of_new.begin(), h.old_of_new.end(), old_of_new_out);
  if (lo_out) std::copy(h.lo.begin(), h.lo.end(), lo_out);
  return GZ_OK;
}

gz_status gz_compile_pattern(const uint8_t* adj, int32_t k, int32_t induced, uint32_t flags,
                             gz_schedule** out) {
  Pattern p;
  if (!read_pattern(adj, k, &p)) return GZ_EINVAL;
  return build_schedule(p, induced, flags, nullptr, out);
}

gz_status gz_compile_pattern_order(const uint8_t* adj, int32_t k, int32_t induced,
                                   const int8_t* order, uint32_t flags, gz_schedule** out) {
  Pattern p;
  if (!read_pattern(adj, k, &p)) return GZ_EINVAL;
  if (!order || !schedule_valid(p, order)) {
    set_error("order is not a valid schedule (a permutation in which every vertex after "
              "the first has an earlier neighbour)");
    return GZ_EINVAL;
  }
  return build_schedule(p, induced, flags, order, out);
}

gz_status gz_schedule_info(const gz_schedule* s, int8_t* order, int8_t* bound,
                           uint64_t* aut_size, int32_t* n_distinct, double* cost) {
  if (!s) {
    set_error("NULL schedule");
    return GZ_EINVAL;
  }
  for (int i = 0; i < kMaxK; ++i) {
    if (order) order[i] = i < s->pat.k ? s->order[i] : -1;
    if (bound) bound[i] = i < s->pat.k ? s->plan.lv[i].bound : -1;
  }
  if (bound && s->pat.k > 0) bound[0] = -1;
  if (aut_size) *aut_size = s->aut_size;
  if (n_distinct) *n_distinct = s->n_distinct;
  if (cost) *cost = s->cost;
  return GZ_OK;
}

gz_status gz_enumerate_schedules(const uint8_t* adj, int32_t k, int32_t induced,
                                 int8_t* orders, double* costs, int32_t max_orders,
                                 int32_t* n_total) {
  Pattern p;
  if (!read_pattern(adj, k, &p)) return GZ_EINVAL;
  if (max_orders > 0 && !orders) {
    set_error("orders is NULL");
    return GZ_EINVAL;
  }
  std::vector<Perm> aut = automorphisms(p);
  std::vector<Perm> ds = explore_schedules(p, aut);
  for (int32_t i = 0; i < (int32_t)ds.size() && i < max_orders; ++i) {
    for (int j = 0; j < kMaxK; ++j) orders[i * kMaxK + j] = j < k ? ds[i][j] : -1;
    if (costs) {
      int8_t b[kMaxK];
      reduced_bounds(p, aut, ds[i].data(), b);
      costs[i] = analytic_cost(p, ds[i].data(), b, induced != 0);
    }
  }
  if (n_total) *n_total = (int32_t)ds.size();
  return GZ_OK;
}

void gz_free_schedule(gz_schedule* s) { delete s; }

static gz_status check_run(const gz_graph* g, const gz_schedule* s) {
  if (!g || !s) {
    set_error("NULL graph or schedule");
    return GZ_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->device) {
    set_error("the current HIP device is not the graph's device");
    return GZ_EINVAL;
  }
  return GZ_OK;
}

gz_status gz_count(const gz_graph* g, const gz_schedule* s, void* hip_stream,
                   uint64_t* out_count) {
  gz_status rc = check_run(g, s);
  if (rc) return rc;
  if (!out_count) {
    set_error("out_count is NULL");
    return GZ_EINVAL;
  }
  unsigned __int128 total = 0;
  rc = run_count(g, s, (hipStream_t)hip_stream, nullptr, 0, nullptr, false, &total, nullptr,
                 nullptr);
  if (rc) return rc;
  if (total >> 64) {
    set_error("count does not fit in 64 bits");
    return GZ_EOVERFLOW;
  }
  *out_count = (uint64_t)total;
  return GZ_OK;
}

gz_status gz_count_noalloc(const gz_graph* g, const gz_schedule* s, void* hip_stream,
                           uint64_t* out_count) {
  gz_status rc = check_run(g, s);
  if (rc) return rc;
  if (!out_count) {
    set_error("NULL output pointer");
    return GZ_EINVAL;
  }
  unsigned __int128 total = 0;
  rc = run_count_noalloc(g, s, (hipStream_t)hip_stream, &total);
  if (rc) return rc;
  if (total >> 64) {
    set_error("count does not fit in 64 bits");
    return GZ_EOVERFLOW;
  }
  *out_count = (uint64_t)total;
  return GZ_OK;
}

gz_status gz_count_timed(const gz_graph* g, const gz_schedule* s, void* hip_stream,
                         uint64_t* out_count, float* kernel_ms) {
  gz_status rc = check_run(g, s);
  if (rc) return rc;
  if (!out_count || !kernel_ms) {
    set_error("NULL output pointer");
    return GZ_EINVAL;
  }
  unsigned __int128 total = 0;
  rc = run_count(g, s, (hipStream_t)hip_stream, nullptr, 0, nullptr, false, &total, nullptr,
                 kernel_ms);
  if (rc) return rc;
  if (total >> 64) {
    set_error("count does not fit in 64 bits");
    return GZ_EOVERFLOW;
  }
  *out_count = (uint64_t)total;
  return GZ_OK;
}

gz_status gz_count_roots(const gz_graph* g, const gz_schedule* s, const int32_t* roots,
                         int64_t n_roots, void* hip_stream, uint64_t* out_per_root) {
  gz_status rc = check_run(g, s);
  if (rc) return rc;
  if (n_roots < 0 || (n_roots > 0 && (!roots || !out_per_root))) {
    set_error("bad root list");
    return GZ_EINVAL;
  }
  for (int64_t i = 0; i < n_roots; ++i)
    if (roots[i] < 0 || roots[i] >= g->host.n) {
      set_error("root id out of range");
      return GZ_EINVAL;
    }
  if (n_roots == 0) return GZ_OK;
  unsigned __int128 total = 0;
  return run_count(g, s, (hipStream_t)hip_stream, roots, n_roots, out_per_root, false, &total,
                   nullptr, nullptr);
}

gz_status gz_count_subset(const gz_graph* g, const gz_schedule* s, const int32_t* roots,
                          int64_t n_roots, void* hip_stream, uint64_t* out_count,
                          float* kernel_ms) {
  gz_status rc = check_run(g, s);
  if (rc) return rc;
  if (!out_count || n_roots < 0 || (n_roots > 0 && !roots)) {
    set_error(out_count ? "bad root list" : "NULL output pointer");
    return GZ_EINVAL;
  }
  for (int64_t i = 0; i < n_roots; ++i)
    if (roots[i] < 0 || roots[i] >= g->host.n) {
      set_error("root id out of range");
      return GZ_EINVAL;
    }
  *out_count = 0;
  if (kernel_ms) *kernel_ms = 0.0f;
  if (n_roots == 0) return GZ_OK;
  unsigned __int128 total = 0;
  rc = run_count(g, s, (hipStream_t)hip_stream, roots, n_roots, nullptr, false, &total, nullptr,
                 kernel_ms);
  if (rc) return rc;
  if (total >> 64) {
    set_error("count does not fit in 64 bits");
    return GZ_EOVERFLOW;
  }
  *out_count = (uint64_t)total;
  return GZ_OK;
}

gz_status gz_count_bytes_subset(const gz_graph* g, const gz_schedule* s, const int32_t* roots,
                                int64_t n_roots, void* hip_stream, uint64_t* out_bytes,
                                uint64_t* out_count) {
  gz_status rc = check_run(g, s);
  if (rc) return rc;
  if (n_roots < 0 || (n_roots > 0 && !roots)) {
    set_error("bad root list");
    return GZ_EINVAL;
  }
  for (int64_t i = 0; i < n_roots; ++i)
    if (roots[i] < 0 || roots[i] >= g->host.n) {
      set_error("root id out of range");
      return GZ_EINVAL;
    }
  unsigned __int128 total = 0, bytes = 0;
  if (n_roots > 0) {
    rc = run_count(g, s, (hipStream_t)hip_stream, roots, n_roots, nullptr, true, &total, &bytes,
                   nullptr);
    if (rc) return rc;
  }
  if ((total >> 64) || (bytes >> 64)) {
    set_error("count or byte total does not fit in 64 bits");
    return GZ_EOVERFLOW;
  }
  if (out_bytes) *out_bytes = (uint64_t)bytes;
  if (out_count) *out_count = (uint64_t)total;
  return GZ_OK;
}

gz_status gz_count_bytes(const gz_graph* g, const gz_schedule* s, void* hip_stream,
                         uint64_t* out_bytes, uint64_t* out_count) {
  gz_status rc = check_run(g, s);
  if (rc) return rc;
  unsigned __int128 total = 0, bytes = 0;
  rc = run_count(g, s, (hipStream_t)hip_stream, nullptr, 0, nullptr, true, &total, &bytes,
                 nullptr);
  if (rc) return rc;
  if ((total >> 64) || (bytes >> 64)) {
    set_error("count or byte total does not fit in 64 bits");
    return GZ_EOVERFLOW;
  }
  if (out_bytes) *out_bytes = (uint64_t)bytes;
  if (out_count) *out_count = (uint64_t)total;
  return GZ_OK;
}

gz_status gz_count_ops(const gz_graph* g, const gz_schedule* s, void* hip_stream,
                       uint64_t* out_ops, uint64_t* out_count) {
  gz_status rc = check_run(g, s);
  if (rc) return rc;
  unsigned __int128 total = 0, ops = 0;
  rc = run_count(g, s, (hipStream_t)hip_stream, nullptr, 0, nullptr, false, &total, &ops, nullptr,
                 true);
  if (rc) return rc;
  if ((total >> 64) || (ops >> 64)) {
    set_error("count or operation total does not fit in 64 bits");
    return GZ_EOVERFLOW;
  }
  if (out_ops) *out_ops = (uint64_t)ops;
  if (out_count) *out_count = (uint64_t)total;
  return GZ_OK;
}

gz_status gz_census_create(const gz_graph* const* graphs, int32_t n_graphs,
                           const gz_schedule* const* scheds, int32_t n_scheds, gz_census** out) {
  return census_create(graphs, n_graphs, scheds, n_scheds, (void**)out);
}

gz_status gz_census_run(gz_census* c, uint64_t* counts, float* ms) {
  if (!c) {
    set_error("NULL census");
    return GZ_EINVAL;
  }
  return census_run(c, counts, ms);
}

gz_status gz_census_tune(gz_census* c, int32_t* params, float* best_ms) {
  if (!c) {
    set_error("NULL census");
    return GZ_EINVAL;
  }
  return census_tune(c, params, best_ms);
}

void gz_census_free(gz_census* c) { census_free(c); }

const char* gz_last_error(void) { return g_last_error.c_str(); }

const char* gz_status_string(gz_status st) {
  switch (st) {
    case GZ_OK: return "ok";
    case GZ_EINVAL: return "invalid argument";
    case GZ_ENOMEM: return "out of memory";
    case GZ_EDEVICE: return "HIP device error";
    case GZ_EOVERFLOW: return "count overflows 64 bits";
    case GZ_ENOTSUP: return "not supported";
    default: return "unknown status";
  }
}

}  // extern "C"
