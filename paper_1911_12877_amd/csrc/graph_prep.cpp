// Host graph preparation: normalisation of raw input into a simple undirected
// CSR with ascending rows, and the degree reindex of GraphZero's generalised
// orientation (Section 6, first technique: higher degree gets a smaller id,
// ties broken by the original id).  Rows stay complete - no edge is pruned -
// and lo[v], the number of neighbours with a smaller id, marks the part of
// each row that a restriction bounded by v itself can reach.
#include <algorithm>
#include <atomic>
#include <thread>

#include "gz_internal.h"

namespace gz {

void parallel_for(int64_t n, int64_t grain,
                  const std::function<void(int64_t, int64_t)>& body) {
  if (n <= 0) return;
  unsigned hw = std::thread::hardware_concurrency();
  int nthreads = (int)std::min<unsigned>(hw ? hw : 1, 16);
  if (n <= grain || nthreads <= 1) {
    body(0, n);
    return;
  }
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    for (;;) {
      int64_t b = next.fetch_add(grain);
      if (b >= n) break;
      body(b, std::min(n, b + grain));
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
}

// Rows of `n` vertices held in `buf` at offsets `off` (length n+1), possibly
// with duplicates: sort, deduplicate and compact into g->rowptr / g->col.
static bool compact_rows(int32_t n, std::vector<int64_t>& off,
                         std::vector<int32_t>& buf, HostGraph* g,
                         std::string* err) {
  std::vector<int64_t> len(n);
  parallel_for(n, 4096, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      int32_t* s = buf.data() + off[v];
      int32_t* t = buf.data() + off[v + 1];
      std::sort(s, t);
      len[v] = std::unique(s, t) - s;
    }
  });
  int64_t total = 0;
  for (int32_t v = 0; v < n; ++v) total += len[v];
  if (total > INT32_MAX) {
    *err = "graph has 2^31 or more neighbour entries";
    return false;
  }
  g->n = n;
  g->rowptr.assign((size_t)n + 1, 0);
  for (int32_t v = 0; v < n; ++v) g->rowptr[v + 1] = g->rowptr[v] + (int32_t)len[v];
  g->col.resize((size_t)total);
  parallel_for(n, 4096, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v)
      std::copy(buf.data() + off[v], buf.data() + off[v] + len[v],
                g->col.data() + g->rowptr[v]);
  });
  g->lo.clear();
  g->old_of_new.clear();
  return true;
}

bool graph_from_edges(const int32_t* src, const int32_t* dst, int64_t m,
                      int32_t n, HostGraph* g, std::string* err) {
  if (n < 0 || m < 0) {
    *err = "negative vertex or edge count";
    return false;
  }
  std::atomic<bool> bad{false};
  parallel_for(m, 1 << 16, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) bad = true;
  });
  if (bad) {
    *err = "edge endpoint out of range [0, n)";
    return false;
  }
  std::vector<int64_t> off((size_t)n + 1, 0);
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] == dst[i]) continue;
    off[src[i] + 1]++;
    off[dst[i] + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  std::vector<int32_t> buf((size_t)off[n]);
  std::vector<int64_t> fill(off.begin(), off.end() - 1);
  for (int64_t i = 0; i < m; ++i) {
    int32_t u = src[i], v = dst[i];
    if (u == v) continue;
    buf[fill[u]++] = v;
    buf[fill[v]++] = u;
  }
  return compact_rows(n, off, buf, g, err);
}

static bool check_csr_shape(const int32_t* rowptr, const int32_t* col, int32_t n,
                            int64_t nnz, std::string* err) {
  if (n < 0 || nnz < 0 || nnz > INT32_MAX) {
    *err = "n or nnz out of range";
    return false;
  }
  if (rowptr[0] != 0 || rowptr[n] != nnz) {
    *err = "rowptr[0] must be 0 and rowptr[n] must equal nnz";
    return false;
  }
  for (int32_t v = 0; v < n; ++v)
    if (rowptr[v + 1] < rowptr[v]) {
      *err = "rowptr is not non-decreasing";
      return false;
    }
  std::atomic<bool> bad{false};
  parallel_for(nnz, 1 << 16, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      if (col[i] < 0 || col[i] >= n) bad = true;
  });
  if (bad) {
    *err = "column index out of range [0, n)";
    return false;
  }
  return true;
}

bool graph_from_csr_normalize(const int32_t* rowptr, const int32_t* col,
                              int32_t n, int64_t nnz, HostGraph* g,
                              std::string* err) {
  if (!check_csr_shape(rowptr, col, n, nnz, err)) return false;
  std::vector<int32_t> src((size_t)nnz);
  parallel_for(n, 4096, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v)
      for (int64_t i = rowptr[v]; i < rowptr[v + 1]; ++i) src[i] = (int32_t)v;
  });
  return graph_from_edges(src.data(), col, nnz, n, g, err);
}

bool graph_from_csr_strict(const int32_t* rowptr, const int32_t* col, int32_t n,
                           int64_t nnz, HostGraph* g, std::string* err) {
  if (!check_csr_shape(rowptr, col, n, nnz, err)) return false;
  std::atomic<int> why{0};
  parallel_for(n, 4096, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      for (int64_t i = rowptr[v]; i < rowptr[v + 1]; ++i) {
        int32_t u = col[i];
        if (u == v) why = 1;
        if (i > rowptr[v] && col[i - 1] >= u) why = 2;
        const int32_t* s = col + rowptr[u];
        const int32_t* t = col + rowptr[u + 1];
        const int32_t* p = std::lower_bound(s, t, (int32_t)v);
        if (p == t || *p != v) why = 3;
      }
    }
  });
  if (why == 1) *err = "self-loop in CSR (use GZ_GRAPH_NORMALIZE)";
  if (why == 2) *err = "CSR rows not strictly ascending (use GZ_GRAPH_NORMALIZE)";
  if (why == 3) *err = "CSR is not symmetric (use GZ_GRAPH_NORMALIZE)";
  if (why) return false;
  g->n = n;
  g->rowptr.assign(rowptr, rowptr + n + 1);
  g->col.assign(col, col + nnz);
  g->lo.clear();
  g->old_of_new.clear();
  return true;
}

void graph_reindex(HostGraph* g) {
  const int32_t n = g->n;
  // counting sort of the vertices by decreasing degree, stable in id
  int32_t maxd = 0;
  for (int32_t v = 0; v < n; ++v) maxd = std::max(maxd, g->rowptr[v + 1] - g->rowptr[v]);
  std::vector<int64_t> start((size_t)maxd + 2, 0);
  for (int32_t v = 0; v < n; ++v) start[maxd - (g->rowptr[v + 1] - g->rowptr[v]) + 1]++;
  for (int32_t d = 0; d <= maxd; ++d) start[d + 1] += start[d];
  std::vector<int32_t> order((size_t)n);
  for (int32_t v = 0; v < n; ++v) order[start[maxd - (g->rowptr[v + 1] - g->rowptr[v])]++] = v;
  std::vector<int32_t> new_of_old((size_t)n);
  for (int32_t r = 0; r < n; ++r) new_of_old[order[r]] = r;

  std::vector<int32_t> rowptr2((size_t)n + 1, 0);
  for (int32_t r = 0; r < n; ++r)
    rowptr2[r + 1] = rowptr2[r] + (g->rowptr[order[r] + 1] - g->rowptr[order[r]]);
  std::vector<int32_t> col2(g->col.size());
  parallel_for(n, 2048, [&](int64_t b, int64_t e) {
    for (int64_t r = b; r < e; ++r) {
      int32_t old = order[r];
      int32_t* out = col2.data() + rowptr2[r];
      int32_t d = g->rowptr[old + 1] - g->rowptr[old];
      const int32_t* in = g->col.data() + g->rowptr[old];
      for (int32_t i = 0; i < d; ++i) out[i] = new_of_old[in[i]];
      std::sort(out, out + d);
    }
  });
  std::vector<int32_t> prev = std::move(g->old_of_new);
  g->old_of_new.resize((size_t)n);
  for (int32_t r = 0; r < n; ++r)
    g->old_of_new[r] = prev.empty() ? order[r] : prev[order[r]];
  g->rowptr = std::move(rowptr2);
  g->col = std::move(col2);
  g->lo.clear();
}

void graph_finish(HostGraph* g) {
  const int32_t n = g->n;
  if (g->old_of_new.empty()) {
    g->old_of_new.resize((size_t)n);
    for (int32_t v = 0; v < n; ++v) g->old_of_new[v] = v;
  }
  g->lo.resize((size_t)n);
  parallel_for(n, 4096, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      const int32_t* s = g->col.data() + g->rowptr[v];
      const int32_t* t = g->col.data() + g->rowptr[v + 1];
      g->lo[v] = (int32_t)(std::lower_bound(s, t, (int32_t)v) - s);
    }
  });
}

}  // namespace gz
