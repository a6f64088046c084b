/*
 * gz.h - C-ABI of the MI355X (gfx950) exact subgraph-counting library.
 *
 * The method is GraphZero's (Mawhirter et al., "GraphZero: Breaking Symmetry
 * for Efficient Graph Mining"): a pattern is compiled into a schedule (an
 * order of its vertices, Section 2.1) plus one symmetry-breaking restriction
 * per loop (Algorithm 1 and Theorem 2), the graph is reindexed so that higher
 * degree means a smaller id (Section 6), and nested loops grow each embedding
 * one vertex at a time by bounded intersections (pattern edges) and
 * subtractions (pattern non-edges) of sorted neighbour lists.  Each instance
 * is counted exactly once (Theorem 1).
 *
 * Conventions
 *  - Every call returns gz_status: GZ_OK (0) or a negative error code; the
 *    calling thread's last error message is available from gz_last_error().
 *    No call aborts the process.
 *  - Input arrays are owned by the caller and only read during the call
 *    (host arrays, or device arrays with GZ_GRAPH_DEVICE_PTRS); nothing is
 *    retained.  Output arrays are caller-provided host buffers.
 *  - Handles are owned by the library until freed.  A graph handle owns its
 *    device memory; both handle types are immutable after creation, so
 *    concurrent gz_count calls on different streams are allowed.
 *  - hip_stream is a hipStream_t (NULL = the default stream); device work of
 *    a call is ordered on that stream and the call returns after it is done.
 *  - Vertex ids are int32, neighbour-array offsets int32 (nnz < 2^31),
 *    counts uint64.
 */
#ifndef GZ_H
#define GZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gz_status;
enum {
    GZ_OK = 0,
    GZ_EINVAL = -1,      /* bad argument, malformed graph or pattern          */
    GZ_ENOMEM = -2,      /* host or device allocation failed                  */
    GZ_EDEVICE = -3,     /* a HIP runtime call failed                          */
    GZ_EOVERFLOW = -4,   /* the exact count does not fit in 64 bits            */
    GZ_ENOTSUP = -5      /* valid request outside what the library handles    */
};

typedef struct gz_graph gz_graph;
typedef struct gz_schedule gz_schedule;

/* ------------------------------------------------------------------ graphs */

/* Flags of gz_load_graph / gz_load_edges. */
#define GZ_GRAPH_NORMALIZE   1u  /* drop self-loops and duplicates, symmetrise,
                                    sort rows; without it the CSR must already
                                    be simple, symmetric and sorted, else
                                    GZ_EINVAL                                 */
#define GZ_GRAPH_NO_REINDEX  2u  /* keep the caller's ids (orientation off);
                                    counts are unchanged, only speed differs  */
#define GZ_GRAPH_DEVICE_PTRS 4u  /* the input arrays are device pointers      */
#define GZ_GRAPH_PREP_DEVICE 8u  /* gz_load_edges only: normalise and reindex
                                    on the device (radix sorts); the result is
                                    identical to the host preparation         */

/*
 * Load a graph given as CSR: rowptr[n+1] (rowptr[0] = 0, non-decreasing,
 * rowptr[n] = nnz) and colidx[nnz] (neighbour ids in [0, n)).  The graph is
 * undirected: each edge {u,v} appears in both rows.  Unless
 * GZ_GRAPH_NO_REINDEX is given, vertices are renumbered by decreasing degree,
 * ties by increasing id (Section 6, first technique); gz_graph_export returns
 * the mapping.  The prepared graph (int32 CSR with ascending rows and, per
 * vertex, the number of neighbours with a smaller id) is uploaded to the
 * current HIP device.  Errors: GZ_EINVAL (n < 0, nnz out of range, malformed
 * CSR), GZ_ENOMEM, GZ_EDEVICE.
 */
gz_status gz_load_graph(const int32_t* rowptr, const int32_t* colidx,
                        int32_t n, int64_t nnz, uint32_t flags,
                        void* hip_stream, gz_graph** out);

/*
 * Load a graph given as a raw edge list src[m], dst[m] over n vertices.  The
 * list may hold self-loops, duplicates and one or both orientations of an
 * edge; it is always normalised (GZ_GRAPH_NORMALIZE is implied).  With
 * GZ_GRAPH_PREP_DEVICE the normalisation and the degree reindex run on the
 * current device (m < 2^31) and the prepared graph is copied back to the
 * handle's host copy; the arrays are the same as those of the host path.
 * Errors: GZ_EINVAL (n < 0, m < 0, an endpoint outside [0, n), a result of
 * 2^31 or more entries, unknown flags), GZ_ENOMEM, GZ_EDEVICE.
 */
gz_status gz_load_edges(const int32_t* src, const int32_t* dst, int64_t m,
                        int32_t n, uint32_t flags, void* hip_stream,
                        gz_graph** out);

/* Sizes of a prepared graph: vertices, stored neighbour entries (twice the
 * edge count), largest degree, largest number of smaller-id neighbours. */
gz_status gz_graph_info(const gz_graph* g, int32_t* n, int64_t* nnz,
                        int32_t* max_deg, int32_t* max_lo_deg);

/* Host copies of the prepared graph: rowptr[n+1], colidx[nnz] and
 * old_of_new[n] (the caller's id of each prepared vertex).  Any pointer may
 * be NULL to skip that array. */
gz_status gz_graph_export(const gz_graph* g, int32_t* rowptr, int32_t* colidx,
                          int32_t* old_of_new);

void gz_free_graph(gz_graph* g);

/*
 * Host-only preparation (no device needed): the same normalisation and
 * degree reindex as gz_load_edges, written to caller buffers.  rowptr_out
 * needs n+1 entries, colidx_out 2*m (an upper bound of the result's nnz),
 * old_of_new_out and lo_out n entries (lo_out[v]: number of neighbours of v
 * with a smaller id).  *nnz_out receives the prepared nnz.  Any of
 * old_of_new_out / lo_out may be NULL.  Errors: GZ_EINVAL for endpoints out
 * of range or a result with 2^31 or more entries.
 */
gz_status gz_prepare_edges(const int32_t* src, const int32_t* dst, int64_t m,
                           int32_t n, uint32_t flags, int64_t* nnz_out,
                           int32_t* rowptr_out, int32_t* colidx_out,
                           int32_t* old_of_new_out, int32_t* lo_out);

/* ---------------------------------------------------------------- patterns */

/* Flags of gz_compile_pattern / gz_compile_pattern_order. */
#define GZ_SCHED_ANALYTIC    0u  /* pick the distinct schedule of lowest
                                    analytic cost (Section 5.4)               */
#define GZ_SCHED_NO_RESTRICT 8u  /* drop all restrictions: every automorphic
                                    mapping is counted, so the result is
                                    |Aut(P)| times the count (Theorem 1);
                                    for tests                                 */

/*
 * Compile a pattern: adj is k*k row-major 0/1, symmetric, zero diagonal,
 * connected, 2 <= k <= 8.  induced != 0 asks for vertex-induced counts (every
 * pattern non-edge must be a graph non-edge, the set subtractions of
 * Section 2.1); induced == 0 counts subgraphs (edge-induced).  Steps: the
 * automorphism group by trying all k! permutations (Section 4.2); the
 * distinct schedules by the explorer (Algorithm 3); per schedule the
 * restrictions (Algorithm 1) reduced to one bound per loop (Theorem 2) and the
 * analytic cost (Section 5.4, appendix); the cheapest schedule is lowered to
 * per-loop descriptors.  Errors: GZ_EINVAL for a malformed or disconnected
 * pattern or k out of range.
 */
gz_status gz_compile_pattern(const uint8_t* adj, int32_t k, int32_t induced,
                             uint32_t flags, gz_schedule** out);

/* Same with a caller-chosen schedule order[k] (a permutation of 0..k-1 in
 * which every vertex after the first has an earlier neighbour).  GZ_EINVAL if
 * the order is not a valid schedule. */
gz_status gz_compile_pattern_order(const uint8_t* adj, int32_t k,
                                   int32_t induced, const int8_t* order,
                                   uint32_t flags, gz_schedule** out);

/*
 * Describe a compiled schedule.  order[8] receives the pattern vertex of each
 * loop; bound[8] the loop whose vertex bounds loop i from above (the graph
 * vertex of loop i must have a smaller id than that of loop bound[i]) or -1;
 * aut_size |Aut(P)|; n_distinct the number of distinct schedules of the
 * pattern; analytic_cost the cost of this schedule.  Any pointer may be NULL.
 */
gz_status gz_schedule_info(const gz_schedule* s, int8_t* order, int8_t* bound,
                           uint64_t* aut_size, int32_t* n_distinct,
                           double* analytic_cost);

/*
 * All distinct schedules of a pattern in the explorer's emission order
 * (Algorithm 3): orders[max_orders*8] receives 8 entries per schedule (the
 * first k used), costs[max_orders] their analytic costs (may be NULL).  At
 * most max_orders are written; *n_total receives the full count.
 */
gz_status gz_enumerate_schedules(const uint8_t* adj, int32_t k,
                                 int32_t induced, int8_t* orders,
                                 double* costs, int32_t max_orders,
                                 int32_t* n_total);

void gz_free_schedule(gz_schedule* s);

/* ---------------------------------------------------------------- counting */

/*
 * Exact number of instances of the compiled pattern in the graph (each
 * instance once; |Aut(P)| times that with GZ_SCHED_NO_RESTRICT).  Runs the
 * mining kernels on hip_stream and waits for them.  Errors: GZ_EINVAL (NULL
 * handle), GZ_EOVERFLOW (count >= 2^64; *out_count is then unspecified),
 * GZ_ENOMEM, GZ_EDEVICE.
 *
 * How the count is evaluated - never its value - can be steered by
 * environment variables read at every call (decimal integers; invalid or
 * out-of-range values are ignored):
 *  - GZ_SPLIT_MIN_LEN (>= 0, default 64) and GZ_SPLIT_CAP (1..2^26,
 *    default 2^22): patterns of k >= 4 on the generic loops run in two
 *    phases; prefixes whose loop base is longer than the threshold are
 *    recorded by the first launch (up to the capacity; later ones are
 *    expanded in place) and expanded in 256-element pieces by a second, the
 *    host reading the record count in between.
 *  - GZ_HUB_MIN_DEG (>= 1, default 512) and GZ_HUB_MAX_KB (KiB, 0 turns
 *    them off, default 32 GiB): the leading vertices of at least that degree
 *    get a dense neighbour bitmap, built on the first count that asks for
 *    it and kept with the graph; membership probes into their lists read
 *    one bit.
 *  - GZ_LONG_MIN (>= 1, default 256), GZ_MERGE_RATIO (eighths, default 4)
 *    and GZ_IE_RATIO (eighths, default 12): last-loop items whose walk
 *    reaches GZ_LONG_MIN elements are counted by a whole wave, merging
 *    probe lists at most GZ_MERGE_RATIO/8 times the walk's length; an item
 *    of a vertex-induced pattern counts by inclusion-exclusion over its
 *    negative lists when that costs less than GZ_IE_RATIO/8 of walking its
 *    shortest positive list.  GZ_IE_FORCE=1 makes every item with negative
 *    lists take inclusion-exclusion.
 *  - GZ_SWEEP_MIN (>= 0, default 16384) and GZ_SWEEP_IE (>= 0, default 2):
 *    when every positive list of the loops before an item's is a hub's, a
 *    group of last-loop items that walk their own rows is swept instead:
 *    those loops' lists become one bit mask per block of 2^15 vertex ids in
 *    LDS, and each item row entry costs one read of the row and one of the
 *    mask.  A group is swept when its rows total at least GZ_SWEEP_MIN
 *    entries (0: never); an item keeps inclusion-exclusion when that walks
 *    under 1/GZ_SWEEP_IE of its row.
 *  - GZ_CLIQUE_MAX_LO (0..1024, default 1024): clique schedules run on
 *    per-root bit rows (see gz_count_ops) for roots with at most this many
 *    first-loop candidates; roots with more take the generic loops.
 *  - GZ_ACC_SEED (test only): the count's 128-bit accumulator (and every
 *    per-root slot of gz_count_roots) starts at this value instead of 0, so
 *    the result is shifted by it; tests drive the overflow checks with it.
 */
gz_status gz_count(const gz_graph* g, const gz_schedule* s, void* hip_stream,
                   uint64_t* out_count);

/*
 * gz_count for callers that cannot allocate device memory (code under HIP
 * graph capture around it, tight serving loops, harnesses that forbid
 * hipMalloc): the same exact count, with no hipMalloc, hipFree or other
 * allocating call.  Its accumulators (16 x 64-bit words) live in a
 * file-scope device array, one copy per GPU held until the process ends;
 * every call on a GPU shares it and clears it first, so calls that overlap
 * on one GPU (any streams) race and must be serialised by the caller.  The
 * graph's first-loop task lists are built when the graph is loaded; the hub
 * bitmaps are used only when an earlier count on the graph built them; long
 * loop bases are expanded in place (no two-phase split).  The launch shape
 * does not depend on the input's size, so no size is rejected.  Errors as
 * gz_count.
 */
gz_status gz_count_noalloc(const gz_graph* g, const gz_schedule* s, void* hip_stream,
                           uint64_t* out_count);

/*
 * gz_count that also reports the mining kernels' own duration in
 * milliseconds, measured with HIP events recorded on hip_stream around the
 * mining launches (both phases and the read-back between them; accumulator
 * set-up and the result copy are outside the interval).
 */
gz_status gz_count_timed(const gz_graph* g, const gz_schedule* s,
                         void* hip_stream, uint64_t* out_count,
                         float* kernel_ms);

/*
 * Per-root counts: out_per_root[i] receives the number of instances whose
 * restricted mapping puts roots[i] (a prepared-graph id) in the first loop.
 * Summed over all vertices these give gz_count.  Errors as gz_count, plus
 * GZ_EINVAL for a root out of range.
 */
gz_status gz_count_roots(const gz_graph* g, const gz_schedule* s,
                         const int32_t* roots, int64_t n_roots,
                         void* hip_stream, uint64_t* out_per_root);

/*
 * Count over a subset of the roots: the number of instances whose restricted
 * mapping puts one of roots[0..n_roots) (prepared-graph ids, none listed
 * twice) in the first loop, with the same kernels and launch shape as
 * gz_count and, when kernel_ms is not NULL, their duration as in
 * gz_count_timed.  Theorem 1 gives every instance exactly one restricted
 * mapping, so the count decomposes exactly over roots: disjoint root sets
 * covering all vertices sum to gz_count.  This is the unit a caller splits
 * one count by (a share of the roots per device, or per step).  Errors as
 * gz_count_roots.
 */
gz_status gz_count_subset(const gz_graph* g, const gz_schedule* s,
                          const int32_t* roots, int64_t n_roots,
                          void* hip_stream, uint64_t* out_count,
                          float* kernel_ms);

/*
 * Algorithmic bytes of one gz_count: over every evaluation of loops 1..k-1,
 * 4 bytes per element of each neighbour list the loop's set expression
 * reads (pattern-edge lists, plus pattern-non-edge lists when induced), cut
 * at the loop's restriction bound (Section 6, second technique), plus 8 bytes
 * per list for its row offsets.  Loop i is evaluated once per iteration of
 * loop i-1, along which only the list of v_{i-1} changes: that list counts
 * per evaluation, the others once per execution of loop i-1 (at its last
 * iteration's cut, the longest).  A loop that extends loop i-1's candidate
 * set reads that set's elements instead of the lists it shares with it.
 * Runs an instrumented (slower) pass; the count of that pass is returned
 * too.
 */
gz_status gz_count_bytes(const gz_graph* g, const gz_schedule* s,
                         void* hip_stream, uint64_t* out_bytes,
                         uint64_t* out_count);

/*
 * gz_count_bytes over a subset of the roots (as in gz_count_subset): the
 * algorithmic bytes of the evaluations reached from the listed roots, and
 * their count.
 */
gz_status gz_count_bytes_subset(const gz_graph* g, const gz_schedule* s,
                                const int32_t* roots, int64_t n_roots,
                                void* hip_stream, uint64_t* out_bytes,
                                uint64_t* out_count);

/*
 * Clique schedules (K_k, 4 <= k <= 8) run on per-root bit rows: row p holds
 * the bounded intersection of the loop after candidate p as a bit set over
 * the root's candidates, and deeper loops AND rows and popcount the result.
 * gz_count_ops runs that path instrumented and returns the number of 32-bit
 * lane operations of those row intersections (each 64-bit row word ANDed
 * costs 2, each 64-bit popcount 2) together with the count.  GZ_ENOTSUP for
 * schedules that do not take the clique path, or when some root has more
 * first-loop candidates than the bit rows hold.
 */
gz_status gz_count_ops(const gz_graph* g, const gz_schedule* s, void* hip_stream,
                       uint64_t* out_ops, uint64_t* out_count);

/* ------------------------------------------------------------ motif census */

/*
 * Batched counting of many patterns (k <= 7) over many graphs in one
 * persistent launch per size class (patterns of 2-5 vertices; of 6-7):
 * every (graph, pattern, first-loop task) item of a class is handed out from
 * one queue, and each (graph, pattern) pair keeps its own 128-bit count.
 * The zeroing of the accumulators and the launches are captured once into a
 * HIP graph and replayed by gz_census_run.  Graph and schedule
 * handles must outlive the census object; counts follow the order
 * counts[graph * n_scheds + sched].  The census runs on its own stream and
 * each call returns when its work is done.  Errors: GZ_EINVAL (NULL or empty
 * inputs, a graph on another device), GZ_ENOTSUP (a pattern of 8 vertices),
 * GZ_ENOMEM, GZ_EDEVICE.
 */
typedef struct gz_census gz_census;

gz_status gz_census_create(const gz_graph* const* graphs, int32_t n_graphs,
                           const gz_schedule* const* scheds, int32_t n_scheds,
                           gz_census** out);

/* One replay; counts[n_graphs * n_scheds] (may be NULL) and the replay's
 * device time in milliseconds (may be NULL).  GZ_EOVERFLOW if a count does
 * not fit in 64 bits. */
gz_status gz_census_run(gz_census* c, uint64_t* counts, float* ms);

/* Autotune the launch: task granularity (first-loop candidates per item) of
 * 3-vertex patterns (8, 32, 128) and of larger ones (1, 4, 16), and items per
 * queue pop (1, 4); defaults before tuning are (128, 1, 1).  Each candidate is
 * rebuilt, captured and replayed twice; the fastest is kept.
 * params[3] receives (granularity k=3, granularity k>=4, items per pop),
 * best_ms its replay time.  Either may be NULL. */
gz_status gz_census_tune(gz_census* c, int32_t* params, float* best_ms);

void gz_census_free(gz_census* c);

/* ------------------------------------------------- learned schedule choice */

/*
 * The analytic model of Section 5.4 assumes a uniform random graph.  A
 * learned cost model can rank the distinct schedules instead: a two-layer
 * perceptron h = relu(W1 x + b1), y = w2 . h + b2 (H hidden units) maps the
 * GZ_FEATURES features of a (schedule, graph) pair to a relative log10 run
 * time.  Parameters are FP32 in one array
 * [W1 (H x D, row-major), b1 (H), w2 (H), b2], GZ_MLP_PARAMS(D, H) floats.
 */
#define GZ_FEATURES 108
#define GZ_MLP_PARAMS(D, H) ((int64_t)(H) * (D) + 2 * (int64_t)(H) + 1)
#define GZ_SCHED_LEARNED 1u   /* gz_compile_pattern_graph: rank by the
                                 installed model (analytic if none)       */

/* Features of the schedule order[k] of a pattern on a prepared graph, into
 * out[GZ_FEATURES] (host).  Per loop 1..7 (zero beyond k): presence, pattern
 * neighbours/7, subtracted non-neighbours/7, bounded, bounded by the
 * previous loop, unbounded with no reusable set, log10 of the loop size in
 * G(n, p) with the graph's n and mean degree (/10), log10 restriction pass
 * rate (/3), last loop, reusable set present, log10 of the loop's
 * cost-model term (/10), intersected and subtracted lists whose owner is
 * itself bounded (/7 each), length of the loop's bound chain (/7) - 14 per
 * loop; then log10 of the whole schedule's cost in this graph's G(n, p) and
 * in the paper's G(1000, 5/999) (/10 each); then graph statistics (log10 of
 * n, edges, mean degree, E[d^2]/E[d], max degree, mean and E[lo^2]/E[lo]
 * and max of the smaller-id degree lo, each scaled).  GZ_EINVAL for a bad
 * pattern/order. */
gz_status gz_schedule_features(const gz_graph* g, const uint8_t* adj, int32_t k,
                               int32_t induced, const int8_t* order,
                               float* out);

/* The last GZ_GRAPH_STATS features of a row are the graph's statistics. */
#define GZ_GRAPH_STATS 8

/* Install (copy) a model for GZ_SCHED_LEARNED, process-wide; params NULL
 * removes it.  D must be GZ_FEATURES, 1 <= H <= 1024.  The learned choice
 * keeps the analytic model's pick unless the network is on known ground
 * and sure:
 *  - margin (log10 of time, >= 0): the network must predict its choice
 *    faster than the analytic pick by more than this;
 *  - k_max (2..8): the largest pattern in its training corpus; larger
 *    patterns keep the analytic pick;
 *  - graph_range (2 x GZ_GRAPH_STATS floats, or NULL for no limit): the
 *    smallest then the largest value of each graph statistic over the
 *    corpus; a graph outside that range (by more than 0.05) keeps the
 *    analytic pick. */
gz_status gz_set_cost_model(const float* params, int32_t D, int32_t H, float margin,
                            int32_t k_max, const float* graph_range);

/* gz_compile_pattern with the graph the schedule will run on.  With
 * GZ_SCHED_LEARNED and an installed model the distinct schedule of lowest
 * predicted cost is chosen (BF16 inference on the current device; ties
 * within 1e-6 go to the explorer's first); otherwise as gz_compile_pattern.
 * The count never depends on the choice (Theorem 1). */
gz_status gz_compile_pattern_graph(const gz_graph* g, const uint8_t* adj,
                                   int32_t k, int32_t induced, uint32_t flags,
                                   gz_schedule** out);

/*
 * MLP kernels on device arrays (hip_stream ordered; the calls wait).
 * gz_mlp_forward: y[n] = model(X[n x D]); bf16 != 0 rounds weights,
 *   inputs and hidden activations to BF16 (FP32 accumulation).
 * gz_mlp_loss_grad: *loss_host = mean((y - t)^2) of the FP32 forward pass and
 *   grad[GZ_MLP_PARAMS] its gradient.
 * gz_mlp_adam: one Adam step (bias-corrected, step >= 1) on params with
 *   moment arrays m, v (same size).
 */
gz_status gz_mlp_forward(const float* params, const float* X, int32_t n, int32_t D,
                         int32_t H, int32_t bf16, float* y, void* hip_stream);
gz_status gz_mlp_loss_grad(const float* params, const float* X, const float* t,
                           int32_t n, int32_t D, int32_t H, float* grad,
                           float* loss_host, void* hip_stream);
gz_status gz_mlp_adam(float* params, const float* grad, float* m, float* v,
                      int32_t D, int32_t H, float lr, float beta1, float beta2,
                      float eps, int32_t step, void* hip_stream);

/* ------------------------------------------------------------------ errors */

const char* gz_last_error(void);
const char* gz_status_string(gz_status status);

#ifdef __cplusplus
}
#endif
#endif /* GZ_H */
