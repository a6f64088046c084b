/*
 * Oracle, counting side: plain single-threaded C.  TEST INFRASTRUCTURE ONLY.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg load it;
 * the product library never links or calls it, and it shares no source with
 * the product.
 *
 * What it computes (the paper's problem statement, Sections 2.1 and 4):
 *   a graph G is simple and undirected; a pattern P has k labelled vertices
 *   and a schedule S (an order of its labels).  A mapping M sends S[0..k-1]
 *   to distinct graph vertices such that every black edge (pattern edge) is
 *   a graph edge and, in vertex-induced mode, every red edge (pattern
 *   non-edge) is a graph non-edge.  With a relation list L (pairs of schedule
 *   positions (a, b), a < b) only mappings with M(S[a]) > M(S[b]) for every
 *   pair are counted (Theorem 1).  With the relations of Algorithm 1 every
 *   instance is counted exactly once; with no relations every instance is
 *   counted |Aut(P)| times.
 *
 * The enumeration is a plain depth-first search over schedule positions.
 * Candidates of position i >= 1 are taken from the neighbour list of one
 * earlier black neighbour (the one of smallest degree), every constraint is
 * then checked one by one, and since rows are sorted the scan stops at the
 * tightest upper bound (Section 6, bounded set operations).
 *
 * Sums are kept in unsigned __int128; callers receive low and high words.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------ graph build */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Simple graph from a raw edge list: drop self-loops, add both directions,
 * sort each row, drop duplicates.  rowptr has n+1 entries; col must hold 2*m
 * entries.  Returns nnz, or -1 on an endpoint out of range. */
int64_t oracle_normalize(int32_t n, int64_t m, const int32_t* src,
                         const int32_t* dst, int64_t* rowptr, int32_t* col) {
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!fill || !deg) { free(fill); free(deg); return -2; }
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = src[e], v = dst[e];
        if (u < 0 || v < 0 || u >= n || v >= n) { free(fill); free(deg); return -1; }
        if (u == v) continue;
        deg[u]++; deg[v]++;
    }
    int64_t* start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int32_t v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v];
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = src[e], v = dst[e];
        if (u == v) continue;
        col[start[u] + fill[u]++] = v;
        col[start[v] + fill[v]++] = u;
    }
    /* sort and deduplicate each row, compacting in place */
    int64_t out = 0;
    rowptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t b = start[v], e = start[v + 1];
        qsort(col + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        for (int64_t i = b; i < e; ++i)
            if (i == b || col[i] != col[i - 1]) col[out++] = col[i];
        rowptr[v + 1] = out;
    }
    free(fill); free(deg); free(start);
    return out;
}

/* Degree reindex (Section 6, first technique): new ids in order of
 * decreasing degree, ties by increasing old id.  new_of_old[v] receives the
 * new id of old vertex v; rowptr2/col2 receive the relabelled graph with
 * sorted rows. */
static const int64_t* g_sort_rowptr;
static int cmp_by_degree(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    int64_t dx = g_sort_rowptr[x + 1] - g_sort_rowptr[x];
    int64_t dy = g_sort_rowptr[y + 1] - g_sort_rowptr[y];
    if (dx != dy) return dx > dy ? -1 : 1;
    return (x > y) - (x < y);
}

void oracle_reindex(int32_t n, const int64_t* rowptr, const int32_t* col,
                    int64_t* rowptr2, int32_t* col2, int32_t* new_of_old) {
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    for (int32_t v = 0; v < n; ++v) order[v] = v;
    g_sort_rowptr = rowptr;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_by_degree);
    for (int32_t r = 0; r < n; ++r) new_of_old[order[r]] = r;
    rowptr2[0] = 0;
    for (int32_t r = 0; r < n; ++r) {
        int32_t old = order[r];
        int64_t d = rowptr[old + 1] - rowptr[old];
        rowptr2[r + 1] = rowptr2[r] + d;
        for (int64_t i = 0; i < d; ++i)
            col2[rowptr2[r] + i] = new_of_old[col[rowptr[old] + i]];
        qsort(col2 + rowptr2[r], (size_t)d, sizeof(int32_t), cmp_i32);
    }
    free(order);
}

/* ------------------------------------------------------------ enumeration */

typedef struct {
    const int64_t* rowptr;
    const int32_t* col;
    int32_t n;
    int k;
    int induced;
    int black[8][8];      /* black[i][j]: schedule positions i, j adjacent */
    int upper[8][8];      /* upper[i][a]: relation (a, i) present, a < i   */
    int32_t m[8];         /* current mapping, by schedule position         */
    u128 count;
    /* instrumentation: one bound per position (Theorem 2 form) */
    int bound[8];
    int extends[8];       /* position i extends position i-1's candidate set */
    int added[8][8];      /* lists position i adds to that set              */
    int32_t rank[8];      /* rank of m[i] among position i's candidates     */
    u128 bytes;
    int instrument;
} search_t;

static int has_edge(const search_t* s, int32_t u, int32_t x) {
    int64_t lo = s->rowptr[u], hi = s->rowptr[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int32_t y = s->col[mid];
        if (y == x) return 1;
        if (y < x) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* |N(u) ∩ [0, b)| by a linear scan of the sorted row */
static int64_t prefix_len(const search_t* s, int32_t u, int64_t b) {
    int64_t c = 0;
    for (int64_t i = s->rowptr[u]; i < s->rowptr[u + 1] && s->col[i] < b; ++i) ++c;
    return c;
}

/* Algorithmic bytes of evaluating position i's candidate set from the
 * current partial mapping m[0..i-1].  Written as a bounded linear merge, the
 * set expression reads, for every earlier position j whose list enters it
 * (black neighbours, and red ones in induced mode), the elements of N(m[j])
 * below the position's bound: 4 bytes each, plus 8 bytes for the list's two
 * row offsets.  When the position extends the candidate set of position i-1
 * (see extension_rule) it reads instead that set's elements below m[i-1]
 * (their number is m[i-1]'s rank in it) and only the lists it adds.
 *
 * Position i is evaluated once per iteration of position i-1's loop, and
 * only N(m[i-1]) changes along that loop: the other operands (the lists of
 * positions before i-1, the extended set) are read once per execution of
 * the loop.  level_bytes_varying counts the per-iteration part (called on
 * entering position i); level_bytes_invariant the rest, once, after position
 * i-1's loop, with m[i-1] and rank[i-1] of its last iteration (the longest
 * cut). */
static int64_t level_cut(const search_t* s, int i) {
    return (s->bound[i] >= 0) ? (int64_t)s->m[s->bound[i]] : INT64_MAX;
}

static int level_reads(const search_t* s, int i, int j) {
    return s->extends[i] ? s->added[i][j] : (s->black[i][j] || s->induced);
}

static void level_bytes_varying(search_t* s, int i) {
    if (level_reads(s, i, i - 1))
        s->bytes += (u128)(4 * prefix_len(s, s->m[i - 1], level_cut(s, i)) + 8);
}

static void level_bytes_invariant(search_t* s, int i) {
    int64_t b = level_cut(s, i);
    if (s->extends[i]) s->bytes += (u128)(4 * (int64_t)s->rank[i - 1]);
    for (int j = 0; j < i - 1; ++j)
        if (level_reads(s, i, j)) s->bytes += (u128)(4 * prefix_len(s, s->m[j], b) + 8);
}

/* Position i (3 <= i <= k-1) extends position i-1's candidate set when it is
 * bounded by position i-1 and every list of position i-1's set expression is
 * also a list of position i's, with the same role (intersected or, in
 * induced mode, subtracted).  Its added lists are the remaining ones. */
static void extension_rule(search_t* s) {
    for (int i = 0; i < s->k; ++i) {
        s->extends[i] = 0;
        for (int j = 0; j < 8; ++j) s->added[i][j] = 0;
    }
    for (int i = 3; i < s->k; ++i) {
        if (s->bound[i] != i - 1) continue;
        int ok = 1;
        for (int j = 0; j < i - 1; ++j) {
            if (s->black[i - 1][j] && !s->black[i][j]) ok = 0;
            if (s->induced && !s->black[i - 1][j] && s->black[i][j]) ok = 0;
        }
        if (!ok) continue;
        s->extends[i] = 1;
        for (int j = 0; j < i; ++j) {
            int in_i = s->black[i][j] || s->induced;
            int in_prev = (j < i - 1) && (s->black[i - 1][j] || s->induced);
            s->added[i][j] = in_i && !in_prev;
        }
    }
}

static void dfs(search_t* s, int i) {
    if (s->instrument) level_bytes_varying(s, i);
    /* source list: the earlier black neighbour of smallest degree */
    int src = -1;
    int64_t best = INT64_MAX;
    for (int j = 0; j < i; ++j) {
        if (!s->black[i][j]) continue;
        int64_t d = s->rowptr[s->m[j] + 1] - s->rowptr[s->m[j]];
        if (d < best) { best = d; src = j; }
    }
    /* tightest upper bound among the relations (a, i) */
    int64_t ub = INT64_MAX;
    for (int a = 0; a < i; ++a)
        if (s->upper[i][a] && s->m[a] < ub) ub = s->m[a];
    int32_t u = s->m[src];
    int32_t accepted = 0, last = 0;
    for (int64_t e = s->rowptr[u]; e < s->rowptr[u + 1]; ++e) {
        int32_t x = s->col[e];
        if (x >= ub) break;
        int ok = 1;
        for (int j = 0; j < i && ok; ++j) {
            if (x == s->m[j]) { ok = 0; break; }
            if (j == src) continue;
            if (s->black[i][j]) ok = has_edge(s, s->m[j], x);
            else if (s->induced) ok = !has_edge(s, s->m[j], x);
        }
        if (!ok) continue;
        if (i == s->k - 1) {
            s->count += 1;
        } else {
            s->m[i] = x;
            s->rank[i] = accepted;
            dfs(s, i + 1);
        }
        last = x;
        ++accepted;
    }
    if (s->instrument && i < s->k - 1 && accepted > 0) {
        s->m[i] = last;
        s->rank[i] = accepted - 1;
        level_bytes_invariant(s, i + 1);
    }
}

static int setup(search_t* s, int32_t n, const int64_t* rowptr, const int32_t* col,
                 int k, const uint8_t* adj, int induced, const int8_t* order,
                 int n_rel, const int8_t* rel_a, const int8_t* rel_b) {
    if (k < 2 || k > 8) return -1;
    memset(s, 0, sizeof(*s));
    s->rowptr = rowptr; s->col = col; s->n = n; s->k = k; s->induced = induced;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            s->black[i][j] = adj[order[i] * k + order[j]] ? 1 : 0;
    for (int i = 1; i < k; ++i) {
        int any = 0;
        for (int j = 0; j < i; ++j) any |= s->black[i][j];
        if (!any) return -2;        /* not a valid schedule */
    }
    for (int r = 0; r < n_rel; ++r) {
        int a = rel_a[r], b = rel_b[r];
        if (a < 0 || b < 0 || a >= k || b >= k || a >= b) return -3;
        s->upper[b][a] = 1;
    }
    for (int i = 0; i < k; ++i) s->bound[i] = -1;
    return 0;
}

/* Count over the roots v0 in roots[0..n_roots) (or over all vertices when
 * roots is NULL).  per_root, when not NULL, receives each root's count
 * (saturating at 2^64-1).  Returns 0, or a negative code on bad input. */
int oracle_count(int32_t n, const int64_t* rowptr, const int32_t* col,
                 int k, const uint8_t* adj, int induced, const int8_t* order,
                 int n_rel, const int8_t* rel_a, const int8_t* rel_b,
                 const int32_t* roots, int64_t n_roots,
                 uint64_t* total_lo, uint64_t* total_hi, uint64_t* per_root) {
    search_t s;
    int rc = setup(&s, n, rowptr, col, k, adj, induced, order, n_rel, rel_a, rel_b);
    if (rc) return rc;
    int64_t cnt = roots ? n_roots : (int64_t)n;
    u128 total = 0;
    for (int64_t r = 0; r < cnt; ++r) {
        int32_t v0 = roots ? roots[r] : (int32_t)r;
        if (v0 < 0 || v0 >= n) return -4;
        s.count = 0;
        s.m[0] = v0;
        dfs(&s, 1);
        total += s.count;
        if (per_root) per_root[r] = (s.count >> 64) ? UINT64_MAX : (uint64_t)s.count;
    }
    *total_lo = (uint64_t)total;
    *total_hi = (uint64_t)(total >> 64);
    return 0;
}

/* Algorithmic bytes of the schedule's bounded set operations (see
 * level_bytes_varying, level_bytes_invariant) summed over every evaluation
 * of positions 1..k-1 reached from the given roots.  bound[i] is the single kept restriction of
 * position i (Theorem 2), -1 for none; the enumeration itself is restricted
 * by exactly these bounds. */
int oracle_instrument(int32_t n, const int64_t* rowptr, const int32_t* col,
                      int k, const uint8_t* adj, int induced, const int8_t* order,
                      const int8_t* bound, const int32_t* roots, int64_t n_roots,
                      uint64_t* bytes_lo, uint64_t* bytes_hi,
                      uint64_t* count_lo, uint64_t* count_hi) {
    int8_t ra[8], rb[8];
    int nr = 0;
    for (int i = 0; i < k; ++i)
        if (bound[i] >= 0) { ra[nr] = bound[i]; rb[nr] = (int8_t)i; ++nr; }
    search_t s;
    int rc = setup(&s, n, rowptr, col, k, adj, induced, order, nr, ra, rb);
    if (rc) return rc;
    for (int i = 0; i < k; ++i) s.bound[i] = bound[i];
    extension_rule(&s);
    s.instrument = 1;
    int64_t cnt = roots ? n_roots : (int64_t)n;
    u128 total = 0;
    for (int64_t r = 0; r < cnt; ++r) {
        int32_t v0 = roots ? roots[r] : (int32_t)r;
        if (v0 < 0 || v0 >= n) return -4;
        s.count = 0;
        s.m[0] = v0;
        dfs(&s, 1);
        total += s.count;
    }
    *bytes_lo = (uint64_t)s.bytes;
    *bytes_hi = (uint64_t)(s.bytes >> 64);
    *count_lo = (uint64_t)total;
    *count_hi = (uint64_t)(total >> 64);
    return 0;
}
