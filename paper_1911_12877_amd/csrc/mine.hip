// HIP mining kernels for gfx950 (wave64): the nested loops of a compiled
// schedule, run as a persistent wave-per-task depth-first search.
//
// Loop 0 enumerates roots v0.  Loop 1's candidates are a contiguous piece of
// N(v0) (its first lo[v0] entries when loop 1 is bounded by v0: the
// orientation prefix); the first-loop work of every root is cut into tasks of
// `chunk` candidates and handed out through an atomic queue in vertex order
// (decreasing degree after reindexing).  Loops 2..k-2 materialise their
// candidate sets in LDS, `CH` base elements at a time; loop k-1 is only
// counted.  A candidate set is the intersection of the neighbour lists of the
// loop's pattern neighbours (Section 2.1), minus the lists of its pattern
// non-neighbours in vertex-induced mode, cut at the loop's single restriction
// bound (Theorem 2) - a prefix of every sorted list (Section 6, bounded set
// operations).  Each set is evaluated from its shortest bounded operand; the
// other operands are probed by binary search, and survivors are compacted
// with ballot + mbcnt.  A loop may instead filter the materialised set of an
// earlier loop whose constraints it contains (plan `src`).
//
// The last loop is flattened: the items of the enclosing loop's chunk are
// laid out one per lane, their base lengths prefix-summed, and every lane
// then takes one (item, base element) pair at a time, so short lists still
// fill the wave.
//
// A prefix whose loop base is longer than a threshold is not expanded by the
// wave that meets it: the wave records it and moves on, and a second launch
// hands the recorded bases out in CH-element pieces, one wave per piece, so a
// hub's list no longer serialises its whole subtree on one wave.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "gz_internal.h"

namespace gz {
namespace dev {

// last-loop items with a shorter walk never try inclusion-exclusion
constexpr int IE_MIN = 256;
constexpr int WAVE = 64;
constexpr int CH = 256;               // base elements per materialised chunk
constexpr int BLOCK = 256;
constexpr int WPB = BLOCK / WAVE;     // waves per workgroup
constexpr int32_t INF = 0x7fffffff;
constexpr int SRC_SLOT = 8;
// walk elements per step of a whole-wave walk: four loads in flight per lane
// for 3- and 4-vertex patterns, fewer for larger ones (registers)
constexpr int WALK_TILE = 4 * WAVE;
template <int K>
constexpr int walk_tile() { return K <= 4 ? WALK_TILE : (K <= 5 ? 2 * WAVE : WAVE); }
// last-loop sweep: an LDS mask covers 2^SW_SHIFT consecutive vertex ids at a
// time; the kernels of patterns up to SW_KMAX vertices carry it
constexpr int SW_SHIFT = 15;
constexpr int SW_WORDS = (1 << SW_SHIFT) / 32;
constexpr int SW_KMAX = 5;
template <int K>
constexpr int sweep_words() { return K <= SW_KMAX ? SW_WORDS : 1; }
// Waves per SIMD the generic kernels are compiled for (1: the compiler's
// choice).  Their loops wait on scattered loads, so for 4-vertex patterns
// more resident waves beat the few registers spilled to reach them.
template <int K>
constexpr int mine_waves() { return K == 4 ? 5 : 1; }
template <int K>
constexpr int heavy_waves() { return K == 4 ? 7 : 1; }

struct Graph {
  const int32_t* __restrict__ rowptr;
  const int32_t* __restrict__ col;
  const int32_t* __restrict__ lo;
  int32_t n;
  // neighbour bitmaps of vertices 0..n_hub-1 (none when n_hub == 0)
  const uint32_t* __restrict__ hub;
  int32_t n_hub;
  long long hub_words;
};

struct HeavyItem;

struct Tasks {
  const int64_t* __restrict__ prefix;  // n_roots + 1
  const int32_t* __restrict__ roots;   // nullptr: root r is vertex r
  const int32_t* __restrict__ slots;   // per-root output slot of root r (nullptr: r)
  int64_t n_roots;
  int64_t n_tasks;
  int32_t chunk;
  int32_t bounded1;                    // loop 1 bounded by v0
  int32_t batch;                       // tasks per queue pop
  int32_t heavy_min;                   // split loop bases longer than this
  HeavyItem* heavy;                    // second-phase list (nullptr: no split)
  long long heavy_cap;
  int32_t queue;                       // acc index of the queue head
};

// acc[0..1]: 128-bit count; acc[2..3]: 128-bit bytes (or operations);
// acc[4]: queue head (k_mine, k_clique_wave); acc[5]: per-root overflow
// flag; acc[6]: split record count; acc[7]: queue head of the generic launch
// over a clique count's roots beyond the bit rows; acc[8..11]: queue heads of
// the clique workgroup launches; per-root counts start at acc[ACC_HEAD]
constexpr int ACC_BLOCK_QUEUES = 8;
constexpr int ACC_HEAD = 16;
struct Out {
  unsigned long long* acc;
  unsigned long long* per_root;
};

template <int K>
struct WaveMem {
  static constexpr int NSET = K >= 4 ? K - 3 : 1;
  int32_t set[NSET][CH];
  int32_t set_len[NSET];
  // The last loop's phases use disjoint LDS: a group's items while their
  // pairs are walked, a merge window during long walks, the sweep mask
  union {
    struct {
      int32_t it_u[WAVE];
      int32_t it_pref[WAVE];
      int32_t it_bstart[WAVE];
      int32_t it_slot[WAVE];
      int32_t it_srclen[WAVE];
      int32_t it_urs[WAVE];
      int32_t it_urd[WAVE];
      int32_t it_ie[WAVE];
      int32_t win[WALK_TILE];  // a window of a list being merged (long walks)
    };
    // one block of the sweep mask: bit x of word w is vertex id base + 32w + x
    uint32_t mask[sweep_words<K>()];
  };
  // the lists of the long walk being counted: start in col, bounded length
  // and owner vertex, by list index (see Lists)
  int32_t ls_start[K];
  int32_t ls_len[K];
  int32_t ls_owner[K];
};

struct Acc {
  unsigned long long cnt;
  unsigned long long bytes;
};

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ int mbcnt(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ int32_t uni(int32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// first index in a[0..len) with a[i] >= x
template <typename P>
__device__ __forceinline__ int lower_bound(P a, int len, int32_t x) {
  int lo = 0;
  while (len > 0) {
    int half = len >> 1;
    if (a[lo + half] < x) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo;
}

template <typename P>
__device__ __forceinline__ bool contains(P a, int len, int32_t x) {
  int i = lower_bound(a, len, x);
  return i < len && a[i] == x;
}

// Is x in the list of v, given as its row cut to the first len entries?
// Every caller probes with an x below the cut's bound (x comes from a list
// cut at the same bound), so membership in the cut is membership in N(v):
// one bit of v's bitmap when v is a hub (in the kernels for large graphs,
// BIG), else a binary search of the cut.
template <bool BIG>
__device__ __forceinline__ bool has_nb(const Graph& g, int32_t v, const int32_t* row, int len,
                                       int32_t x) {
  if (BIG && v < g.n_hub)
    return (g.hub[(long long)v * g.hub_words + (x >> 5)] >> (x & 31)) & 1u;
  return contains(row, len, x);
}

// number of entries of the row (start, deg) below bound B; `own` when B is
// the row's own vertex, whose smaller-id part has length lo
__device__ __forceinline__ int bounded_len(const Graph& g, int32_t v, int32_t start,
                                           int32_t deg, int32_t B, bool own) {
  if (B == INF) return deg;
  if (own) return g.lo[v];
  return lower_bound(g.col + start, deg, B);
}

__device__ __forceinline__ int wave_excl_scan(int x, int* total) {
  const int lane = lane_id();
  int v = x;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    int y = __shfl_up(v, d, WAVE);
    if (lane >= d) v += y;
  }
  *total = __shfl(v, WAVE - 1, WAVE);
  return v - x;
}

// ------------------------------------------------------------ last loop

// How many x of the sorted walk W[0..lw) lie in every list of `pos`, in no
// list of `neg`, in the materialised set src[0..src_len) when src_len >= 0,
// and differ from the owners of the lists in `exm` - the whole wave taking
// walk_tile<K>() consecutive elements of W at a time (coalesced, up to
// four loads in flight per lane).  The lists are those of one last-loop evaluation, held
// in the wave's LDS (ls_start, ls_len, ls_owner: index j < K - 2 is loop
// j's row, K - 2 the item's own row, each cut to its bounded length).  A
// probe list at most ratio8 / 8 times as long as the walk is merged: the
// wave streams it forward a tile of entries at a time through an LDS window
// alongside the walk, each window holding the entries up to the tile's
// largest element, and every lane binary-searches the window; longer lists
// (a hub's row beside a short walk) are probed per element, by bitmap or
// binary search.  The result is wave-uniform.
template <int K, bool BIG>
__device__ long long wave_walk(const Graph& g, WaveMem<K>& M, const int32_t* W, int lw,
                               uint32_t pos, uint32_t neg, const int32_t* src, int src_len,
                               uint32_t exm, int ratio8) {
  constexpr int TILE = walk_tile<K>();
  constexpr int U = TILE / WAVE;
  const int lane = lane_id();
  uint32_t mer = 0;
  int pc[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    pc[j] = 0;
    if ((((pos | neg) >> j) & 1u) && 8ll * M.ls_len[j] <= (long long)ratio8 * lw) mer |= 1u << j;
  }
  long long cnt = 0;
  for (int t0 = 0; t0 < lw; t0 += TILE) {
    int32_t x[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = t0 + u * WAVE + lane;
      ok[u] = idx < lw;
      x[u] = ok[u] ? W[idx] : INF;
    }
    const int32_t xmax = W[min(t0 + TILE, lw) - 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int j = 0; j < K; ++j)
        if ((exm >> j) & 1u) ok[u] = ok[u] && x[u] != M.ls_owner[j];
      if (ok[u] && src_len >= 0) ok[u] = contains(src, src_len, x[u]);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (!(((pos | neg) >> j) & 1u)) continue;
      const int32_t* P = g.col + M.ls_start[j];
      const int plen = M.ls_len[j];
      const bool want = ((pos >> j) & 1u) != 0;
      bool in[U];
#pragma unroll
      for (int u = 0; u < U; ++u) in[u] = false;
      if ((mer >> j) & 1u) {
        for (;;) {
          int c = 0;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int q = pc[j] + u * WAVE + lane;
            const int32_t y = q < plen ? P[q] : INF;
            c += __popcll(__ballot(y <= xmax));
            M.win[u * WAVE + lane] = y;
          }
          wave_sync();
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (ok[u] && !in[u]) in[u] = contains(M.win, c, x[u]);
          wave_sync();
          pc[j] += c;
          if (c < TILE) break;
        }
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (ok[u]) in[u] = has_nb<BIG>(g, M.ls_owner[j], P, plen, x[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) ok[u] = ok[u] && (in[u] == want);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) cnt += __popcll(__ballot(ok[u]));
  }
  return cnt;
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t x) {
#pragma unroll
  for (int d = WAVE / 2; d >= 1; d >>= 1) x = min(x, __shfl_xor(x, d, WAVE));
  return uni(x);
}

// Last-loop sweep over one group of items, one per lane (`mine` where the
// lane's item takes part).  Each item walks its own row g.col[start ..
// start + len) (already cut to the loop's bound), and an entry x counts when
// it lies in every list of `pm`, in no list of `nm` (lists of the loops
// before the item's) and differs from the vertices of the loops in `em`.
// Those tests do not depend on the item, so they are folded into one bit
// mask over vertex ids, built in LDS a block of 2^SW_SHIFT ids at a time:
// AND of the positive lists' hub bitmaps, AND-NOT of the negative lists'
// (a negative list without a bitmap clears its entries' bits), the `em`
// vertices cleared.  Every entry then costs one coalesced read of its row
// and one LDS read, instead of one scattered bitmap probe per list.  Blocks
// no item reaches are skipped.  Within a block the items' runs are read a
// tile of 64 consecutive entries at a time, up to SW_TILES tiles of
// different items in flight.  The result is wave-uniform.
constexpr int SW_TILES = 8;
template <int K>
__device__ long long sweep_items(const Graph& g, WaveMem<K>& M, const int32_t (&v)[K],
                                 const int32_t (&rs)[K], const int32_t (&rd)[K], uint32_t pm,
                                 uint32_t nm, uint32_t em, bool mine, int32_t start,
                                 int32_t len) {
  const int lane = lane_id();
  int c = 0;  // the lane's item: entries before c are done
  // its next entry, or a placeholder below the block's end while a whole
  // tile of the item fell in the current block
  int32_t nx = (mine && len > 0) ? g.col[start] : INF;
  int pc[K];  // cursors of the negative lists without a bitmap
#pragma unroll
  for (int j = 0; j < K; ++j) pc[j] = 0;
  long long cnt = 0;
  for (;;) {
    const int32_t m0 = wave_min_i32(nx);
    if (m0 == INF) break;
    const int32_t base = m0 & ~((1 << SW_SHIFT) - 1);
    const long long top = (long long)base + (1 << SW_SHIFT);
    const long long w0 = base >> 5;
#pragma unroll 2
    for (int w = lane; w < SW_WORDS; w += WAVE) {
      const bool in_row = w0 + w < g.hub_words;
      uint32_t m = ~0u;
      if (in_row) {
#pragma unroll
        for (int j = 0; j < K - 2; ++j) {
          if ((pm >> j) & 1u) m &= g.hub[(long long)v[j] * g.hub_words + w0 + w];
          if (((nm >> j) & 1u) && v[j] < g.n_hub) m &= ~g.hub[(long long)v[j] * g.hub_words + w0 + w];
        }
      } else if (pm != 0u) {
        m = 0u;  // ids past the graph's last vertex
      }
      M.mask[w] = m;
    }
    wave_sync();
#pragma unroll
    for (int j = 0; j < K - 2; ++j) {
      if (!((nm >> j) & 1u) || v[j] < g.n_hub) continue;
      for (;;) {
        const int q = pc[j] + lane;
        const int32_t y = q < rd[j] ? g.col[rs[j] + q] : INF;
        const bool below = y < top;
        if (below && y >= base) atomicAnd(&M.mask[(y - base) >> 5], ~(1u << (y & 31)));
        const int adv = __popcll(__ballot(below));
        pc[j] += adv;
        if (adv < WAVE) break;
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < K - 2; ++j)
        if (((em >> j) & 1u) && v[j] >= base && v[j] < top)
          atomicAnd(&M.mask[(v[j] - base) >> 5], ~(1u << (v[j] & 31)));
    }
    wave_sync();
    for (;;) {
      unsigned long long act = __ballot(nx < top);
      if (act == 0ull) break;
      int it[SW_TILES];
      int32_t x[SW_TILES];
#pragma unroll
      for (int u = 0; u < SW_TILES; ++u) {
        it[u] = -1;
        x[u] = INF;
        if (act != 0ull) {
          it[u] = __ffsll((long long)act) - 1;
          act &= act - 1;
          const int ci = __builtin_amdgcn_readlane(c, it[u]);
          const int li = __builtin_amdgcn_readlane(len, it[u]);
          const int32_t si = __builtin_amdgcn_readlane(start, it[u]);
          const int q = ci + lane;
          x[u] = q < li ? g.col[si + q] : INF;
        }
      }
#pragma unroll
      for (int u = 0; u < SW_TILES; ++u) {
        if (it[u] < 0) continue;
        const bool in = x[u] < top;
        const int wi = in ? (x[u] - base) >> 5 : 0;
        const bool ok = in && ((M.mask[wi] >> (x[u] & 31)) & 1u);
        cnt += __popcll(__ballot(ok));
        const int adv = __popcll(__ballot(in));
        // the item's first entry past the block (INF past its row's end)
        const int32_t after = adv < WAVE ? __builtin_amdgcn_readlane(x[u], adv) : 0;
        if (lane == it[u]) {
          c += adv;
          nx = adv < WAVE ? after : (c < len ? base : INF);
        }
      }
    }
    wave_sync();
  }
  return cnt;
}

// Count of the last loop for the items of one chunk of loop K-2.
//
// Each item's candidates are x < B in every positive list (the loop's
// pattern neighbours, or the materialised `src` set plus the rest) and in no
// negative list (pattern non-neighbours, vertex-induced mode), x distinct
// from the `excl` vertices.  Two evaluations give the same number:
//  * direct: walk the shortest bounded positive list and probe the others;
//  * inclusion-exclusion over the negative lists N_1..N_m:
//      sum over T of (-1)^|T| |(all positive lists) and (N_j, j in T)|,
//    each term walked from its own shortest bounded list, less the excl
//    vertices that pass every test.  An item takes it when its unit cost
//    (walked elements times the lists probed per element) is lower: a
//    hub's long positive list is then never walked when its negative lists
//    are short.
// Items whose walk is short share the wave: every (item, term, element)
// pair is one lane's work.  Items with a long walk are counted one at a time
// by the whole wave (wave_walk).  An item's terms are all counted within this
// call, so the signed partial sums of the call total the (non-negative)
// count of its items.
template <int K, bool INSTR, bool IE, bool BIG>
__device__ void last_level(const Graph& g, const Plan& plan, WaveMem<K>& M,
                           const int32_t (&v)[K], const int32_t (&rs)[K],
                           const int32_t (&rd)[K], uint32_t complete,
                           const int32_t* items, int n_items, Acc& acc) {
  constexpr int J = K - 2;  // loop of the items
  const Level L = plan.lv[K - 1];
  const int lane = lane_id();
  const bool use_src = L.src >= 0 && ((complete >> L.src) & 1u);
  const int src_idx = use_src ? L.src - 2 : 0;
  const uint32_t pos = use_src ? L.pos_src : L.isect;
  const uint32_t neg = use_src ? L.neg_src : L.sub;
  const bool item_bound = (L.bound == J);
  const int32_t Bu = (L.bound >= 0 && !item_bound) ? v[L.bound] : INF;
  const int32_t* srcset = M.set[src_idx];
  const int src_full = use_src ? M.set_len[src_idx] : 0;
  const int n_pos = __popc(pos) + (use_src ? 1 : 0);
  const int m_neg = __popc(neg);
  // items walking their own row may be swept instead (sweep_items): the
  // lists of the earlier loops must then be tests of the entry alone - every
  // positive one a hub's bitmap
  bool sweep_on = false;
  uint32_t sw_pm = 0u, sw_nm = 0u, sw_em = 0u;
  if constexpr (BIG && !INSTR && K <= SW_KMAX) {
    const uint32_t early = (1u << J) - 1u;
    if (plan.sweep_min > 0 && !plan.ie_force && !use_src && ((pos >> J) & 1u) &&
        !((neg >> J) & 1u)) {
      sw_pm = pos & early;
      sw_nm = neg & early;
      sw_em = L.excl & early;
      sweep_on = true;
#pragma unroll
      for (int j = 0; j < J; ++j)
        if (((sw_pm >> j) & 1u) && v[j] >= g.n_hub) sweep_on = false;
    }
  }

  // bounded lengths of the rows of loops j < J (exact when the bound does
  // not depend on the item; otherwise the full row, an upper bound that is
  // still correct for membership probes)
  int ulen[K];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    ulen[j] = 0;
    if (((pos | neg) >> j) & 1u)
      ulen[j] = item_bound ? rd[j] : bounded_len(g, v[j], rs[j], rd[j], Bu, L.bound == j);
  }

  long long local = 0;  // signed: inclusion-exclusion terms subtract
  for (int g0 = 0; g0 < n_items; g0 += WAVE) {
    const int t = g0 + lane;
    const bool valid = t < n_items;
    const int32_t u = valid ? items[t] : 0;
    const int32_t urs = valid ? g.rowptr[u] : 0;
    const int32_t urd = valid ? g.rowptr[u + 1] - urs : 0;
    const int32_t B = item_bound ? u : Bu;
    int slot = SRC_SLOT, blen = INF, bstart = 0, slen = 0;
    int len[K];  // bounded length of each list of the loop (j <= J)
#pragma unroll
    for (int j = 0; j < K; ++j) len[j] = 0;
    bool ie = false;
    long long ie_walk = 0;
    if (valid) {
      if (use_src) {
        slen = (L.src == J && item_bound) ? t : lower_bound(srcset, src_full, B);
        blen = slen;
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if ((pos >> j) & 1u) {
          len[j] = item_bound ? lower_bound(g.col + rs[j], rd[j], B) : ulen[j];
          if (len[j] < blen) {
            blen = len[j];
            slot = j;
            bstart = rs[j];
          }
        }
      }
      if ((pos >> J) & 1u) {
        len[J] = bounded_len(g, u, urs, urd, B, item_bound);
        if (len[J] < blen) {
          blen = len[J];
          slot = J;
          bstart = urs;
        }
      }
      if constexpr (INSTR) {
        // the item's own list (the lists of the earlier loops, and the
        // enclosing set an extension reads, stay the same along the items'
        // loop: invariant_bytes, once per execution of that loop)
        const bool ext = (L.acct & 0x80u) != 0;
        const uint32_t all = ext ? (L.acct & 0x7fu) : (uint32_t)(L.isect | L.sub);
        if ((all >> J) & 1u)
          acc.bytes += 4ull * (unsigned)bounded_len(g, u, urs, urd, B, item_bound) + 8ull;
      } else if (IE && m_neg > 0 && (plan.ie_force || blen > IE_MIN || BIG)) {
#pragma unroll
        for (int j = 0; j < J; ++j)
          if ((neg >> j) & 1u)
            len[j] = item_bound ? lower_bound(g.col + rs[j], rd[j], B) : ulen[j];
        if ((neg >> J) & 1u) len[J] = bounded_len(g, u, urs, urd, B, item_bound);
        // unit costs (one per walked element and per probe of it): direct
        // walks the base and probes every other list; inclusion-exclusion
        // walks the base with the positive lists only (not at all when it
        // is the only one) and each term's shortest list with the term's
        // lists as positive ones
        long long& cost = ie_walk;
        long long ie_cost = n_pos > 1 ? (long long)blen * n_pos : 0;
        for (uint32_t T = 1; T < (1u << m_neg); ++T) {
          int mn = blen;
          uint32_t rest = neg;
          for (int q = 0; q < m_neg; ++q) {
            const int j = __ffs(rest) - 1;
            rest &= rest - 1;
            if ((T >> q) & 1u) mn = min(mn, len[j]);
          }
          cost += mn;
          ie_cost += (long long)mn * (n_pos + __popc(T));
        }
        const long long direct_cost = (long long)blen * (n_pos + m_neg);
        ie = plan.ie_force ||
             (blen > IE_MIN && 8 * ie_cost < (long long)plan.ie_ratio * direct_cost);
      }
    } else {
      blen = 0;
    }
    // swept items: walking their own row, unless inclusion-exclusion walks
    // less than 1 / sweep_ie of it; a group sweeps when the swept walks
    // total at least sweep_min entries (the mask's cost is per block)
    bool sw = false;
    if constexpr (BIG && !INSTR && K <= SW_KMAX) {
      if (sweep_on) {
        const long long ie_all = (n_pos > 1 ? blen : 0) + ie_walk;
        sw = valid && slot == J && blen > 0 &&
             (!ie || (long long)plan.sweep_ie * ie_all >= (long long)blen);
        long long tot = sw ? blen : 0;
#pragma unroll
        for (int d = WAVE / 2; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, WAVE);
        if (tot < plan.sweep_min) sw = false;
        if (sw) ie = false;
      }
    }
    // items with a long walk are counted by the whole wave below, 64
    // consecutive elements at a time; the rest share the wave pair by pair
    const long long walk = ie ? (n_pos > 1 ? blen : 0) + ie_walk : (sw ? 0 : blen);
    const bool lng = BIG && !INSTR && valid && walk >= plan.long_min;
    const bool any_ie = IE && __ballot(ie && !lng) != 0ull;
    const uint32_t n_terms = any_ie ? (1u << m_neg) : 1u;
    M.it_u[lane] = u;
    M.it_srclen[lane] = slen;
    M.it_urs[lane] = urs;
    M.it_urd[lane] = urd;
    M.it_ie[lane] = ie ? 1 : 0;
    for (uint32_t T = 0; T < n_terms; ++T) {
      // the term's lists: the positive ones and the negative ones picked by T
      uint32_t tmask = 0;
      {
        uint32_t rest = neg;
        for (int q = 0; q < m_neg; ++q) {
          const int j = __ffs(rest) - 1;
          rest &= rest - 1;
          if ((T >> q) & 1u) tmask |= 1u << j;
        }
      }
      int elen = 0, eslot = slot, estart = bstart;
      if (lng) {
        elen = 0;
      } else if (!ie) {
        elen = (T == 0 && !sw) ? blen : 0;
      } else if (T == 0) {
        if (n_pos == 1) local += blen;  // a single bounded list: its length
        else elen = blen;
      } else {
        elen = blen;
        for (int j = 0; j <= J; ++j) {
          if (((tmask >> j) & 1u) && len[j] < elen) {
            elen = len[j];
            eslot = j;
            estart = (j == J) ? urs : rs[j];
          }
        }
      }
      int total;
      const int pref = wave_excl_scan(elen, &total);
      M.it_pref[lane] = pref;
      M.it_bstart[lane] = estart;
      M.it_slot[lane] = eslot;
      wave_sync();
      const int nvalid = min(WAVE, n_items - g0);
      const long long sign = (__popc(T) & 1) ? -1ll : 1ll;
      for (int p0 = 0; p0 < total; p0 += WAVE) {
        const int p = p0 + lane;
        bool ok = p < total;
        if (ok) {
          // item of pair p: the last i with pref[i] <= p
          int lo = 0, hi = nvalid;
          while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (M.it_pref[mid] <= p) lo = mid + 1; else hi = mid;
          }
          const int i = lo - 1;
          const int e = p - M.it_pref[i];
          const int sl = M.it_slot[i];
          const int32_t x = (sl == SRC_SLOT) ? srcset[e] : g.col[M.it_bstart[i] + e];
          const int32_t uu = M.it_u[i];
          const bool direct = M.it_ie[i] == 0;
          if (direct) {
#pragma unroll
            for (int j = 0; j < J; ++j)
              if ((L.excl >> j) & 1u) ok = ok && (x != v[j]);
            if ((L.excl >> J) & 1u) ok = ok && (x != uu);
          }
          if (ok && use_src && sl != SRC_SLOT) ok = contains(srcset, M.it_srclen[i], x);
#pragma unroll
          for (int j = 0; j < J; ++j)
            if (ok && (((pos | tmask) >> j) & 1u) && sl != j)
              ok = has_nb<BIG>(g, v[j], g.col + rs[j], ulen[j], x);
          if (ok && (((pos | tmask) >> J) & 1u) && sl != J)
            ok = has_nb<BIG>(g, uu, g.col + M.it_urs[i], M.it_urd[i], x);
          if (direct) {
#pragma unroll
            for (int j = 0; j < J; ++j)
              if (ok && ((neg >> j) & 1u)) ok = !has_nb<BIG>(g, v[j], g.col + rs[j], ulen[j], x);
            if (ok && ((neg >> J) & 1u)) ok = !has_nb<BIG>(g, uu, g.col + M.it_urs[i], M.it_urd[i], x);
          }
        }
        local += ok ? sign : 0ll;
      }
      wave_sync();
    }
    // long walks: one item at a time over the whole wave
    if constexpr (BIG) {
      for (unsigned long long lm = __ballot(lng); lm; lm &= lm - 1) {
        const int i = __ffsll((long long)lm) - 1;
        const int32_t ui = uni(__shfl(u, i, WAVE)), ursi = uni(__shfl(urs, i, WAVE));
        const int sloti = uni(__shfl(slot, i, WAVE)), bleni = uni(__shfl(blen, i, WAVE));
        const int bstarti = uni(__shfl(bstart, i, WAVE)), sleni = uni(__shfl(slen, i, WAVE));
        const bool iei = uni(__shfl(ie ? 1 : 0, i, WAVE)) != 0;
        // the item's lists, into the wave's LDS
        {
          // bounded lengths: the item's own, from its lane
          int32_t st = 0, ow = 0, ln = 0;
#pragma unroll
          for (int j = 0; j <= J; ++j) {
            const int32_t lj = __shfl(len[j], i, WAVE);
            if (lane == j) {
              st = (j == J) ? ursi : rs[j];
              ow = (j == J) ? ui : v[j];
              ln = lj;
            }
          }
          if (lane < K) {
            M.ls_start[lane] = st;
            M.ls_len[lane] = ln;
            M.ls_owner[lane] = ow;
          }
        }
        wave_sync();
        const uint32_t nt = iei ? (1u << m_neg) : 1u;
        for (uint32_t T = 0; T < nt; ++T) {
          uint32_t tmask = 0;
          {
            uint32_t rest = neg;
            for (int q = 0; q < m_neg; ++q) {
              const int j = __ffs(rest) - 1;
              rest &= rest - 1;
              if ((T >> q) & 1u) tmask |= 1u << j;
            }
          }
          // the term's walk: the base list, or a shorter list of the term
          int es = sloti, el = bleni;
          if (iei && T > 0) {
            for (int j = 0; j <= J; ++j)
              if (((tmask >> j) & 1u) && M.ls_len[j] < el) {
                el = M.ls_len[j];
                es = j;
              }
          }
          long long c;
          if (iei && T == 0 && n_pos == 1) {
            c = bleni;  // a single bounded list: its length
          } else {
            const int32_t* Wp = (es == SRC_SLOT) ? srcset
                                : g.col + (es == sloti ? bstarti : M.ls_start[es]);
            const uint32_t pm = (pos | tmask) & ~(es == SRC_SLOT ? 0u : (1u << es));
            c = wave_walk<K, BIG>(g, M, Wp, el, pm, iei ? 0u : neg, srcset,
                                  (use_src && es != SRC_SLOT) ? sleni : -1,
                                  iei ? 0u : (uint32_t)L.excl, plan.merge_ratio);
          }
          if (lane == 0) local += (__popc(T) & 1) ? -c : c;
        }
        wave_sync();  // the item's lists stay in LDS until its terms are done
      }
    }
    if constexpr (BIG && !INSTR && K <= SW_KMAX) {
      if (sweep_on && __ballot(sw) != 0ull) {
        const long long c = sweep_items<K>(g, M, v, rs, rd, sw_pm, sw_nm, sw_em, sw, urs, blen);
        if (lane == 0) local += c;
      }
    }
    if (ie) {
      // inclusion-exclusion counted the excl vertices that pass every test
      for (int j = 0; j <= J; ++j) {
        if (!((L.excl >> j) & 1u)) continue;
        const int32_t y = (j == J) ? u : v[j];
        bool ok = y < B;
        if (ok && use_src) ok = contains(srcset, slen, y);
        for (int jj = 0; jj < J; ++jj)
          if (ok && ((pos >> jj) & 1u)) ok = has_nb<BIG>(g, v[jj], g.col + rs[jj], ulen[jj], y);
        if (ok && ((pos >> J) & 1u)) ok = has_nb<BIG>(g, u, g.col + urs, urd, y);
        for (int jj = 0; jj < J; ++jj)
          if (ok && ((neg >> jj) & 1u)) ok = !has_nb<BIG>(g, v[jj], g.col + rs[jj], ulen[jj], y);
        if (ok && ((neg >> J) & 1u)) ok = !has_nb<BIG>(g, u, g.col + urs, urd, y);
        local -= ok ? 1ll : 0ll;
      }
    }
  }
  // the call's items are complete: their signed partial sums total >= 0
#pragma unroll
  for (int d = WAVE / 2; d >= 1; d >>= 1) local += __shfl_xor(local, d, WAVE);
  if (lane == 0) acc.cnt += (unsigned long long)local;
}

// ---------------------------------------------------- materialised loops

// A prefix (v_0..v_{I-1}) whose loop-I base is long is not expanded by the
// wave that meets it; it is recorded and its base later handed out in
// CH-element pieces, one wave per piece (second phase).
struct HeavyItem {
  int32_t v[kMaxK - 1];
  int32_t level;
  int32_t r;         // root slot (per-root mode)
  int32_t base_len;
};

struct Split {
  HeavyItem* items;              // nullptr: never split
  unsigned long long* n_items;   // atomic count (may exceed cap: then not split)
  long long cap;
  int min_len;                   // split bases longer than this
  int32_t r;                     // current root slot
};

// Algorithmic bytes of loop I's set expression that do not change along the
// loop above it (loop I-1): the lists of the loops before I-1 or, when loop
// I extends loop I-1's set, that set's elements below v[I-1] and the lists it
// adds before I-1.  They are counted once per execution of loop I-1, at its
// last iteration (v[I-1] its last element, of rank `rank_last`), whose cut
// is the longest.  The list of v[I-1] itself is counted per iteration.
template <int K, int I>
__device__ unsigned long long invariant_bytes(const Graph& g, const Level& L,
                                              const int32_t (&v)[K], const int32_t (&rs)[K],
                                              const int32_t (&rd)[K], int rank_last) {
  const int32_t B = L.bound >= 0 ? v[L.bound] : INF;
  const bool ext = (L.acct & 0x80u) != 0;
  const uint32_t all = ext ? (L.acct & 0x7fu) : (uint32_t)(L.isect | L.sub);
  unsigned long long b = ext ? 4ull * (unsigned)rank_last : 0ull;
#pragma unroll
  for (int j = 0; j < I - 1; ++j)
    if ((all >> j) & 1u)
      b += 4ull * (unsigned)bounded_len(g, v[j], rs[j], rd[j], B, L.bound == j) + 8ull;
  return b;
}

template <int K, int I, bool INSTR, bool IE, bool BIG>
__device__ void mat_level(const Graph& g, const Plan& plan, WaveMem<K>& M,
                          int32_t (&v)[K], int32_t (&rs)[K], int32_t (&rd)[K],
                          uint32_t complete, Acc& acc, const Split& sp,
                          int c_lo = 0, int c_hi = INF) {
  const Level L = plan.lv[I];
  const int lane = lane_id();
  const int32_t B = L.bound >= 0 ? v[L.bound] : INF;
  if (INSTR && lane == 0) {
    // the list of v[I-1], per evaluation (the rest: invariant_bytes)
    const bool ext = (L.acct & 0x80u) != 0;
    const uint32_t all = ext ? (L.acct & 0x7fu) : (uint32_t)(L.isect | L.sub);
    if ((all >> (I - 1)) & 1u)
      acc.bytes +=
          4ull * (unsigned)bounded_len(g, v[I - 1], rs[I - 1], rd[I - 1], B, L.bound == I - 1) + 8ull;
  }
  const bool use_src = L.src >= 0 && ((complete >> L.src) & 1u);
  const int src_idx = use_src ? L.src - 2 : 0;
  const int32_t* srcset = M.set[src_idx];
  const int src_len = use_src ? lower_bound(srcset, M.set_len[src_idx], B) : 0;
  const uint32_t pos = use_src ? L.pos_src : L.isect;
  const uint32_t neg = use_src ? L.neg_src : L.sub;

  int blen = use_src ? src_len : INF, slot = SRC_SLOT, bstart = 0;
  int len[K];
#pragma unroll
  for (int j = 0; j < I; ++j) {
    len[j] = 0;
    if (((pos | neg) >> j) & 1u) len[j] = bounded_len(g, v[j], rs[j], rd[j], B, L.bound == j);
    if (((pos >> j) & 1u) && len[j] < blen) {
      blen = len[j];
      slot = j;
      bstart = rs[j];
    }
  }
  blen = uni(blen);
  if (!INSTR && sp.items && !use_src && c_lo == 0 && c_hi == INF && blen > sp.min_len) {
    unsigned long long q = 0;
    if (lane == 0) q = atomicAdd(sp.n_items, 1ull);
    q = __shfl(q, 0, WAVE);
    if ((long long)q < sp.cap) {
      if (lane == 0) {
        HeavyItem& it = sp.items[q];
#pragma unroll
        for (int j = 0; j < I; ++j) it.v[j] = v[j];
        it.level = I;
        it.r = sp.r;
        it.base_len = blen;
      }
      return;
    }
  }
  slot = uni(slot);
  bstart = uni(bstart);

  int32_t* out = M.set[I - 2];
  uint32_t mine = complete & ~(1u << I);
  const int c_end = min(blen, c_hi);
  if (blen <= CH && c_lo == 0) mine |= 1u << I;
  int cum = 0;  // survivors of earlier chunks: rank of this chunk's first element
  int32_t last = 0;  // the last survivor so far
  for (int c0 = c_lo; c0 < c_end; c0 += CH) {
    const int c1 = min(c_end, c0 + CH);
    int nout = 0;
    for (int r = c0; r < c1; r += WAVE) {
      const int idx = r + lane;
      bool ok = idx < c1;
      int32_t x = 0;
      if (ok) x = (slot == SRC_SLOT) ? srcset[idx] : g.col[bstart + idx];
#pragma unroll
      for (int j = 0; j < I; ++j)
        if ((L.excl >> j) & 1u) ok = ok && (x != v[j]);
      if (ok && use_src && slot != SRC_SLOT) ok = contains(srcset, src_len, x);
#pragma unroll
      for (int j = 0; j < I; ++j)
        if (ok && ((pos >> j) & 1u) && slot != j) ok = has_nb<BIG>(g, v[j], g.col + rs[j], len[j], x);
#pragma unroll
      for (int j = 0; j < I; ++j)
        if (ok && ((neg >> j) & 1u)) ok = !has_nb<BIG>(g, v[j], g.col + rs[j], len[j], x);
      const unsigned long long m = __ballot(ok);
      if (ok) out[nout + mbcnt(m)] = x;
      nout += __popcll(m);
    }
    if (lane == 0) M.set_len[I - 2] = nout;
    wave_sync();
    if (INSTR && nout > 0) last = uni(out[nout - 1]);
    if constexpr (I == K - 2) {
      last_level<K, INSTR, IE, BIG>(g, plan, M, v, rs, rd, mine, out, nout, acc);
    } else {
      for (int t = 0; t < nout; ++t) {
        v[I] = uni(out[t]);
        rs[I] = uni(g.rowptr[v[I]]);
        rd[I] = uni(g.rowptr[v[I] + 1]) - rs[I];
        mat_level<K, I + 1, INSTR, IE, BIG>(g, plan, M, v, rs, rd, mine, acc, sp);
      }
    }
    cum += nout;
    wave_sync();
  }
  if (INSTR && cum > 0) {
    v[I] = last;
    if (lane == 0) acc.bytes += invariant_bytes<K, I + 1>(g, plan.lv[I + 1], v, rs, rd, cum - 1);
  }
}

// --------------------------------------------------------------- kernels

__device__ __forceinline__ void add_u128(unsigned long long* lo_hi,
                                         unsigned long long lo,
                                         unsigned long long hi) {
  unsigned long long old = atomicAdd(lo_hi, lo);
  if (old + lo < old) hi += 1;
  if (hi) atomicAdd(lo_hi + 1, hi);
}

// 128-bit sum over the wave of one 64-bit value per lane, on lane 0
__device__ __forceinline__ void wave_sum_u128(unsigned long long x,
                                              unsigned long long* lo,
                                              unsigned long long* hi) {
  unsigned long long a = x & 0xffffffffull, b = x >> 32;
#pragma unroll
  for (int d = WAVE / 2; d >= 1; d >>= 1) {
    a += __shfl_xor(a, d, WAVE);
    b += __shfl_xor(b, d, WAVE);
  }
  // x_total = b * 2^32 + a, with a, b < 2^38
  unsigned long long l = a + (b << 32);
  unsigned long long h = (b >> 32) + (l < a ? 1ull : 0ull);
  *lo = l;
  *hi = h;
}

template <int K, bool PER_ROOT, bool INSTR, bool IE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(mine_waves<K>())))
void k_mine(Graph g, Plan plan, Tasks T, Out o) {
  __shared__ WaveMem<K> mem[WPB];
  WaveMem<K>& M = mem[threadIdx.x / WAVE];
  const int lane = lane_id();
  Acc acc{0ull, 0ull};
  int32_t v[K], rs[K], rd[K];
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = rs[j] = rd[j] = 0;

  for (;;) {
    long long t0 = 0;
    if (lane == 0) t0 = (long long)atomicAdd(o.acc + T.queue, (unsigned long long)T.batch);
    t0 = __shfl(t0, 0, WAVE);
    if (t0 >= T.n_tasks) break;
    const long long t1 = min(t0 + (long long)T.batch, T.n_tasks);
    for (long long t = t0; t < t1; ++t) {
      // root of task t: the last r with prefix[r] <= t
      long long lo = 0, hi = T.n_roots + 1;
      while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if (T.prefix[mid] <= t) lo = mid + 1; else hi = mid;
      }
      const long long r = lo - 1;
      const long long slot = T.slots ? T.slots[r] : r;
      const int32_t v0 = uni(T.roots ? T.roots[r] : (int32_t)r);
      const int32_t rs0 = uni(g.rowptr[v0]);
      const int32_t rd0 = uni(g.rowptr[v0 + 1]) - rs0;
      const int32_t len1 = T.bounded1 ? uni(g.lo[v0]) : rd0;
      const int32_t begin = (int32_t)(t - T.prefix[r]) * T.chunk;
      const int32_t end = min(begin + T.chunk, len1);
      v[0] = v0;
      rs[0] = rs0;
      rd[0] = rd0;
      if constexpr (K == 2) {
        if (lane == 0) acc.cnt += (unsigned long long)(end - begin);
      } else if constexpr (K == 3) {
        last_level<K, INSTR, IE, (K <= 7)>(g, plan, M, v, rs, rd, 0u, g.col + rs0 + begin,
                                           end - begin, acc);
      } else {
        for (int32_t i = begin; i < end; ++i) {
          v[1] = uni(g.col[rs0 + i]);
          rs[1] = uni(g.rowptr[v[1]]);
          rd[1] = uni(g.rowptr[v[1] + 1]) - rs[1];
          const Split sp{T.heavy, o.acc + 6, T.heavy_cap, T.heavy_min, (int32_t)slot};
          mat_level<K, 2, INSTR, IE, (K <= 7)>(g, plan, M, v, rs, rd, 0u, acc, sp);
        }
      }
      if constexpr (INSTR && K >= 3) {
        // loop 2's lists of v0: once per root, with the root's last loop-1 element
        if (end == len1 && len1 > 0) {
          v[1] = uni(g.col[rs0 + len1 - 1]);
          if (lane == 0) acc.bytes += invariant_bytes<K, 2>(g, plan.lv[2], v, rs, rd, len1 - 1);
        }
      }
      if constexpr (PER_ROOT) {
        unsigned long long l, h;
        wave_sum_u128(acc.cnt, &l, &h);
        if (lane == 0) {
          unsigned long long old = atomicAdd(o.per_root + slot, l);
          if (h || old + l < old) atomicOr(o.acc + 5, 1ull);
        }
        acc.cnt = 0;
      }
    }
  }
  unsigned long long l, h;
  wave_sum_u128(acc.cnt, &l, &h);
  if (lane == 0 && (l | h)) add_u128(o.acc, l, h);
  if (INSTR) {
    wave_sum_u128(acc.bytes, &l, &h);
    if (lane == 0 && (l | h)) add_u128(o.acc + 2, l, h);
  }
}

// ------------------------------------------------------ clique fast path
//
// K_k (k >= 4) with its chain of bounds (every loop below the previous one):
// the loops after v0 only ever intersect the candidates with lists of
// vertices that are themselves candidates, all inside C1 = N(v0) ∩ [0, v0)
// (the first lo[v0] entries of v0's row).  So C1 is staged in LDS once per
// root and its adjacency stored as bit rows: bit q of row p says that C1[q]
// (smaller than C1[p]) is a neighbour of C1[p], i.e. row p is the bounded
// intersection C1 ∩ N(C1[p]) ∩ [0, C1[p]) of the loop after C1[p].  Every
// deeper bounded intersection is then an AND of rows and the last loop a
// popcount.  Roots with at most 64 candidates run one wave per root with a
// single word per row; larger ones run one workgroup per root with multi-word
// rows in dynamic LDS.

struct RootList {
  const int32_t* __restrict__ v;  // root vertices
  const int32_t* __restrict__ r;  // output slot of each root (per-root mode)
  long long n;
};

constexpr int CW = 64;
constexpr int CBLOCK = 512;            // workgroup path: 8 waves per root
constexpr int CWPB = CBLOCK / WAVE;

struct CliqueWaveMem {
  int32_t xs[CW];
  unsigned long long rows[CW];
  int32_t pref[CW];
  int32_t slot[CW];
  int32_t urs[CW];
  int32_t ulen[CW];
};

// Cliques with D+1 more vertices inside AND(rows[ids[0..n)]) restricted to
// words [0, nw): for D == 0 the popcount, otherwise a sum over the set's
// members b, descending into rows[b] (whose bits all lie below b).
template <int D, bool IN>
__device__ unsigned long long cl_count(const unsigned long long* rows, int W, int (&ids)[8],
                                       int n, int nw, unsigned long long& ops) {
  unsigned long long total = 0;
  for (int w = 0; w < nw; ++w) {
    unsigned long long s = ~0ull;
    for (int t = 0; t < n; ++t) s &= rows[ids[t] * W + w];
    // instrumented: 32-bit lane ops of this word's ANDs and final popcount
    if (IN) ops += 2ull * (unsigned)(n - 1) + (D == 0 ? 2ull : 0ull);
    if constexpr (D == 0) {
      total += (unsigned long long)__popcll(s);
    } else {
      while (s) {
        const int b = w * 64 + __builtin_ctzll(s);
        s &= s - 1;
        ids[n] = b;
        total += cl_count<D - 1, IN>(rows, W, ids, n + 1, w + 1, ops);
      }
    }
  }
  return total;
}

// Position of the r-th (0-based) set bit of x, which has more than r set
// bits: halving by popcount, six steps.
__device__ __forceinline__ int select64(unsigned long long x, int r) {
  int pos = 0;
  int c = __popc((unsigned int)x);
  if (r >= c) {
    r -= c;
    x >>= 32;
    pos = 32;
  }
  c = __popc((unsigned int)x & 0xFFFFu);
  if (r >= c) {
    r -= c;
    x >>= 16;
    pos += 16;
  }
  c = __popc((unsigned int)x & 0xFFu);
  if (r >= c) {
    r -= c;
    x >>= 8;
    pos += 8;
  }
  c = __popc((unsigned int)x & 0xFu);
  if (r >= c) {
    r -= c;
    x >>= 4;
    pos += 4;
  }
  c = __popc((unsigned int)x & 0x3u);
  if (r >= c) {
    r -= c;
    x >>= 2;
    pos += 2;
  }
  if (r >= (int)(x & 1u)) pos += 1;
  return pos;
}

// 5-cliques of the root through the edge (C1[a], C1[b]), b < a, b in word
// wb: the sum over c in m = row a AND row b of popcount(m AND row c).  The
// first four words of m stay in registers, so each c costs one LDS read per
// word in the common case instead of three; members are scanned in 32-bit
// halves, since the kernel is bound by VALU issue and 64-bit bit scans and
// clears take twice the instructions.
__device__ __forceinline__ unsigned long long k5_edge(const unsigned long long* rows, int W,
                                                      int a, int b, int wb) {
  const unsigned long long* ra = rows + (size_t)a * W;
  const unsigned long long* rb = rows + (size_t)b * W;
  const unsigned long long m0 = ra[0] & rb[0];
  const unsigned long long m1 = wb >= 1 ? (ra[1] & rb[1]) : 0ull;
  const unsigned long long m2 = wb >= 2 ? (ra[2] & rb[2]) : 0ull;
  const unsigned long long m3 = wb >= 3 ? (ra[3] & rb[3]) : 0ull;
  unsigned int total = 0;  // at most |C1|^2 members per edge
  for (int wc = 0; wc <= wb; ++wc) {
    const unsigned long long mw = wc == 0 ? m0 : wc == 1 ? m1 : wc == 2 ? m2 : wc == 3 ? m3
                                                                             : (ra[wc] & rb[wc]);
    // members in 32-bit halves: bit scans and clears stay 32-bit
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      unsigned int mc = half ? (unsigned int)(mw >> 32) : (unsigned int)mw;
      const int cbase = wc * 64 + half * 32;
      // two members c per iteration: their row loads are independent
      while (mc) {
        const int c1 = cbase + __builtin_ctz(mc);
        mc &= mc - 1;
        const bool two = mc != 0u;
        const int c2 = two ? cbase + __builtin_ctz(mc) : c1;
        if (two) mc &= mc - 1;
        const unsigned long long* r1 = rows + (size_t)c1 * W;
        const unsigned long long* r2 = rows + (size_t)c2 * W;
        unsigned int n1 = (unsigned)__popcll(m0 & r1[0]);
        unsigned int n2 = (unsigned)__popcll(m0 & r2[0]);
        if (wc >= 1) {
          n1 += (unsigned)__popcll(m1 & r1[1]);
          n2 += (unsigned)__popcll(m1 & r2[1]);
        }
        if (wc >= 2) {
          n1 += (unsigned)__popcll(m2 & r1[2]);
          n2 += (unsigned)__popcll(m2 & r2[2]);
        }
        if (wc >= 3) {
          n1 += (unsigned)__popcll(m3 & r1[3]);
          n2 += (unsigned)__popcll(m3 & r2[3]);
        }
        for (int j = 4; j <= wc; ++j) {
          const unsigned long long m = ra[j] & rb[j];
          n1 += (unsigned)__popcll(m & r1[j]);
          n2 += (unsigned)__popcll(m & r2[j]);
        }
        total += n1 + (two ? n2 : 0u);
      }
    }
  }
  return total;
}

// K-cliques of the root that take C1[a] as their second vertex and a member
// of word w of row a as their third
template <int K, bool IN>
__device__ __forceinline__ unsigned long long clique_unit(const unsigned long long* rows, int W,
                                                         int a, int w, unsigned long long& ops) {
  int ids[8];
  ids[0] = a;
  unsigned long long s = rows[a * W + w];
  unsigned long long total = 0;
  while (s) {
    const int b = w * 64 + __builtin_ctzll(s);
    s &= s - 1;
    ids[1] = b;
    total += cl_count<K - 4, IN>(rows, W, ids, 2, w + 1, ops);
  }
  return total;
}

// Probe plan of row p: slot 0 probes C1[0..p) into N+(C1[p]) (binary search
// in global memory); slot 1 scans N+(C1[p]) and probes each element into
// C1[0..p) (binary search in LDS, most misses rejected by a filter first) -
// the scan is taken unless N+(C1[p]) is more than twice as long (the
// threshold measured fastest on R-MAT scale 20 among 1, 2, 4 and 16).
__device__ __forceinline__ void row_plan(const Graph& g, int32_t x, int p, int32_t* urs,
                                         int32_t* ulen, int32_t* slot, int* len) {
  const int32_t lx = g.lo[x];
  *urs = g.rowptr[x];
  *ulen = lx;
  const bool scan = lx <= 2 * p;
  *slot = scan ? 1 : 0;
  *len = scan ? lx : p;
}

__device__ __forceinline__ int row_probe(const Graph& g, const int32_t* xs, int a, int e,
                                         int32_t slot, int32_t urs, int32_t ulen) {
  if (slot == 0) return contains(g.col + urs, ulen, xs[e]) ? e : -1;
  const int32_t y = g.col[urs + e];
  const int q = lower_bound(xs, a, y);
  return (q < a && xs[q] == y) ? q : -1;
}

// Wave path: roots with at most 64 candidates.
template <int K, bool PER_ROOT, bool IN>
__global__ __launch_bounds__(BLOCK) void k_clique_wave(Graph g, RootList L, Out o, int batch) {
  __shared__ CliqueWaveMem mem[WPB];
  CliqueWaveMem& M = mem[threadIdx.x / WAVE];
  const int lane = lane_id();
  unsigned long long cnt = 0, ops = 0;
  for (;;) {
    long long t0 = 0;
    if (lane == 0) t0 = (long long)atomicAdd(o.acc + 4, (unsigned long long)batch);
    t0 = __shfl(t0, 0, WAVE);
    if (t0 >= L.n) break;
    const long long t1 = min(t0 + (long long)batch, L.n);
    for (long long t = t0; t < t1; ++t) {
      const int32_t v0 = uni(L.v[t]);
      const int d = uni(g.lo[v0]);
      if (d >= K - 1) {
        const int32_t rs0 = uni(g.rowptr[v0]);
        int len = 0;
        if (lane < d) {
          M.xs[lane] = g.col[rs0 + lane];
          row_plan(g, M.xs[lane], lane, &M.urs[lane], &M.ulen[lane], &M.slot[lane], &len);
        }
        M.rows[lane] = 0ull;
        int total;
        M.pref[lane] = wave_excl_scan(len, &total);
        wave_sync();
        for (int p0 = 0; p0 < total; p0 += WAVE) {
          const int p = p0 + lane;
          if (p < total) {
            int lo2 = 0, hi2 = d;
            while (lo2 < hi2) {
              int mid = (lo2 + hi2) >> 1;
              if (M.pref[mid] <= p) lo2 = mid + 1; else hi2 = mid;
            }
            const int a = lo2 - 1;
            const int bit = row_probe(g, M.xs, a, p - M.pref[a], M.slot[a], M.urs[a], M.ulen[a]);
            if (bit >= 0) atomicOr(&M.rows[a], 1ull << bit);
          }
        }
        wave_sync();
        if (lane < d) cnt += clique_unit<K, IN>(M.rows, 1, lane, 0, ops);
        wave_sync();
      }
      if constexpr (PER_ROOT) {
        unsigned long long l, h;
        wave_sum_u128(cnt, &l, &h);
        if (lane == 0) {
          unsigned long long old = atomicAdd(o.per_root + L.r[t], l);
          if (h || old + l < old) atomicOr(o.acc + 5, 1ull);
        }
        cnt = 0;
      }
    }
  }
  if constexpr (!PER_ROOT) {
    unsigned long long l, h;
    wave_sum_u128(cnt, &l, &h);
    if (lane == 0 && (l | h)) add_u128(o.acc, l, h);
  }
  if constexpr (IN) {
    unsigned long long l, h;
    wave_sum_u128(ops, &l, &h);
    if (lane == 0 && (l | h)) add_u128(o.acc + 2, l, h);
  }
}

// Workgroup path: roots with more than 64 candidates (at most 64 W).
// Dynamic LDS: rows[S*W] (64-bit) then xs, pref, urs, ulen, slot (S int32
// each), S = 64 W, then a FILT_BITS-bit membership filter of C1: most
// scanned neighbours are not in C1 and are rejected by one filter read
// instead of a binary search.
constexpr int FILT_BITS = 1 << 15;
constexpr int FILT_WORDS = FILT_BITS / 32;

__device__ __forceinline__ uint32_t filt_hash(int32_t y) {
  return ((uint32_t)y * 0x9E3779B1u) >> 17;  // 15 bits, multiplicative
}

template <int K, bool PER_ROOT, bool IN>
__global__ __launch_bounds__(CBLOCK) void k_clique_block(Graph g, RootList L, Out o, int W,
                                                         unsigned long long* queue) {
  extern __shared__ unsigned long long dyn[];
  __shared__ int s_task;
  __shared__ int s_tot[CWPB];
  const int S = 64 * W;
  unsigned long long* rows = dyn;
  int32_t* xs = (int32_t*)(rows + (size_t)S * W);
  int32_t* pref = xs + S;
  int32_t* urs = pref + S;
  int32_t* ulen = urs + S;
  int32_t* slot = ulen + S;
  uint32_t* filt = (uint32_t*)(slot + S);
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / WAVE;
  unsigned long long cnt = 0, ops = 0;
  for (;;) {
    if (tid == 0) s_task = (int)atomicAdd(queue, 1ull);
    __syncthreads();
    const long long t = s_task;
    __syncthreads();
    if (t >= L.n) break;
    const int32_t v0 = L.v[t];
    const int d = g.lo[v0];
    const int32_t rs0 = g.rowptr[v0];
    const int Wd = (d + 63) / 64;
    for (int q = tid; q < d * Wd; q += CBLOCK) rows[(q / Wd) * W + (q % Wd)] = 0ull;
    for (int q = tid; q < FILT_WORDS; q += CBLOCK) filt[q] = 0u;
    __syncthreads();
    // probe lengths of the rows and their exclusive prefix over the block
    const int per = (d + CBLOCK - 1) / CBLOCK;
    int mysum = 0;
    for (int j = 0; j < per; ++j) {
      const int a = tid * per + j;
      if (a < d) {
        const int32_t x = g.col[rs0 + a];
        xs[a] = x;
        const uint32_t hx = filt_hash(x);
        atomicOr(&filt[hx >> 5], 1u << (hx & 31));
        int len;
        row_plan(g, x, a, &urs[a], &ulen[a], &slot[a], &len);
        // rows of at least a wave's length are probed one wave per row
        // (coalesced, no search for the row); the others are flattened
        const int flat = len < WAVE ? len : 0;
        if (len >= WAVE) slot[a] |= 2;
        pref[a] = flat;
        mysum += flat;
      }
    }
    int wtot;
    const int wexcl = wave_excl_scan(mysum, &wtot);
    if (lane == 0) s_tot[wv] = wtot;
    __syncthreads();
    int base = 0, total = 0;
    for (int w2 = 0; w2 < CWPB; ++w2) {
      if (w2 < wv) base += s_tot[w2];
      total += s_tot[w2];
    }
    int run = base + wexcl;
    for (int j = 0; j < per; ++j) {
      const int a = tid * per + j;
      if (a < d) {
        const int l = pref[a];
        pref[a] = run;
        run += l;
      }
    }
    __syncthreads();
    for (int a = wv; a < d; a += CWPB) {
      const int sl = slot[a];
      if (!(sl & 2)) continue;
      const int len = (sl & 1) ? ulen[a] : a;
      for (int e = lane; e < len; e += WAVE) {
        int bit = -1;
        if (!(sl & 1)) {
          bit = contains(g.col + urs[a], ulen[a], xs[e]) ? e : -1;
        } else {
          const int32_t y = g.col[urs[a] + e];
          const uint32_t hy = filt_hash(y);
          if ((filt[hy >> 5] >> (hy & 31)) & 1u) {
            const int q = lower_bound(xs, a, y);
            bit = (q < a && xs[q] == y) ? q : -1;
          }
        }
        if (bit >= 0) atomicOr(&rows[a * W + (bit >> 6)], 1ull << (bit & 63));
      }
    }
    // short rows: (row, element) pairs flattened over the block; rows of
    // length 0 in the prefix (the long ones) are never the last row at or
    // below a pair's index
    for (int p = tid; p < total; p += CBLOCK) {
      int lo2 = 0, hi2 = d;
      while (lo2 < hi2) {
        int mid = (lo2 + hi2) >> 1;
        if (pref[mid] <= p) lo2 = mid + 1; else hi2 = mid;
      }
      const int a = lo2 - 1;
      const int e = p - pref[a];
      int bit = -1;
      if (slot[a] == 0) {
        bit = contains(g.col + urs[a], ulen[a], xs[e]) ? e : -1;
      } else {
        const int32_t y = g.col[urs[a] + e];
        const uint32_t hy = filt_hash(y);
        if ((filt[hy >> 5] >> (hy & 31)) & 1u) {
          const int q = lower_bound(xs, a, y);
          bit = (q < a && xs[q] == y) ? q : -1;
        }
      }
      if (bit >= 0) atomicOr(&rows[a * W + (bit >> 6)], 1ull << (bit & 63));
    }
    __syncthreads();
    unsigned long long mine = 0;
    if constexpr (K == 4) {
      for (int q = tid; q < d * Wd; q += CBLOCK) {
        const int a = q / Wd, w = q - a * Wd;
        if (w * 64 < a) mine += clique_unit<K, IN>(rows, W, a, w, ops);
      }
    } else {
      // Units are the edges (a, b), b < a, of the candidates' subgraph in
      // row-major order, dealt round-robin (EG consecutive edges per unit; 1
      // measured fastest of 1, 2, 4, 8 for K5 on R-MAT scale 20):
      // the deeper loops' cost varies far more between rows than between
      // edges.  pref[a] becomes the exclusive prefix of the rows' edge counts.
      int es = 0;
      for (int j = 0; j < per; ++j) {
        const int a = tid * per + j;
        if (a < d) {
          int c = 0;
          for (int w = 0; w < Wd; ++w) c += __popcll(rows[a * W + w]);
          pref[a] = c;
          es += c;
        }
      }
      int etot;
      const int eexcl = wave_excl_scan(es, &etot);
      __syncthreads();
      if (lane == 0) s_tot[wv] = etot;
      __syncthreads();
      int ebase = 0, E = 0;
      for (int w2 = 0; w2 < CWPB; ++w2) {
        if (w2 < wv) ebase += s_tot[w2];
        E += s_tot[w2];
      }
      int erun = ebase + eexcl;
      for (int j = 0; j < per; ++j) {
        const int a = tid * per + j;
        if (a < d) {
          const int c = pref[a];
          pref[a] = erun;
          erun += c;
        }
      }
      __syncthreads();
      constexpr int EG = 1;
      for (int e0 = tid * EG; e0 < E; e0 += CBLOCK * EG) {
        const int e1 = min(E, e0 + EG);
        // the row holding edge e0: the last a with pref[a] <= e0 (non-empty)
        int lo2 = 0, hi2 = d;
        while (lo2 < hi2) {
          const int mid = (lo2 + hi2) >> 1;
          if (pref[mid] <= e0) lo2 = mid + 1; else hi2 = mid;
        }
        int a = lo2 - 1;
        int r = e0 - pref[a];
        int w = 0;
        unsigned long long word = rows[a * W];
        for (;;) {
          const int c = __popcll(word);
          if (r < c) break;
          r -= c;
          ++w;
          word = rows[a * W + w];
        }
        word &= ~0ull << select64(word, r);  // drop the r lowest members
        for (int e = e0; e < e1; ++e) {
          while (word == 0) {  // next word of row a (bits lie below a), else next row
            if (++w * 64 >= a) {
              ++a;
              w = 0;
            }
            word = rows[a * W + w];
          }
          const int b = w * 64 + __builtin_ctzll(word);
          word &= word - 1;
          if constexpr (K == 5 && !IN) {
            mine += k5_edge(rows, W, a, b, w);
          } else {
            int ids[8];
            ids[0] = a;
            ids[1] = b;
            mine += cl_count<K - 4, IN>(rows, W, ids, 2, w + 1, ops);
          }
        }
      }
    }
    if constexpr (PER_ROOT) {
      unsigned long long l, h;
      wave_sum_u128(mine, &l, &h);
      if (lane == 0 && (l | h)) {
        unsigned long long old = atomicAdd(o.per_root + L.r[t], l);
        if (h || old + l < old) atomicOr(o.acc + 5, 1ull);
      }
    } else {
      cnt += mine;
    }
    __syncthreads();
  }
  if constexpr (!PER_ROOT) {
    unsigned long long l, h;
    wave_sum_u128(cnt, &l, &h);
    if (lane == 0 && (l | h)) add_u128(o.acc, l, h);
  }
  if constexpr (IN) {
    unsigned long long l, h;
    wave_sum_u128(ops, &l, &h);
    if (lane == 0 && (l | h)) add_u128(o.acc + 2, l, h);
  }
}

// Second phase: the bases of recorded prefixes of one loop depth LV, CH
// elements per item; item t names a record through an exclusive prefix over
// the records' piece counts.  Pieces do not share materialised sets, so the
// loops below take their operands from the neighbour lists.  One launch per
// depth keeps one chain of loops per kernel.
template <int K, bool PER_ROOT, int LV, bool IE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(heavy_waves<K>())))
void k_mine_heavy(Graph g, Plan plan, const HeavyItem* items,
                                                      const long long* piece_prefix,
                                                      long long n_items,
                                                      unsigned long long* queue, Out o) {
  __shared__ WaveMem<K> mem[WPB];
  WaveMem<K>& M = mem[threadIdx.x / WAVE];
  const int lane = lane_id();
  const long long total = piece_prefix[n_items];
  const Split none{nullptr, nullptr, 0, INF, 0};
  Acc acc{0ull, 0ull};
  for (;;) {
    long long t = 0;
    if (lane == 0) t = (long long)atomicAdd(queue, 1ull);
    t = __shfl(t, 0, WAVE);
    if (t >= total) break;
    long long lo = 0, hi = n_items + 1;
    while (lo < hi) {
      long long mid = (lo + hi) >> 1;
      if (piece_prefix[mid] <= t) lo = mid + 1; else hi = mid;
    }
    const long long h = lo - 1;
    const HeavyItem& it = items[h];
    int32_t v[K], rs[K], rd[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      v[j] = (j < LV) ? uni(it.v[j]) : 0;
      rs[j] = (j < LV) ? uni(g.rowptr[v[j]]) : 0;
      rd[j] = (j < LV) ? uni(g.rowptr[v[j] + 1]) - rs[j] : 0;
    }
    const int c0 = (int)(t - piece_prefix[h]) * CH;
    mat_level<K, LV, false, IE, (K <= 7)>(g, plan, M, v, rs, rd, 0u, acc, none, c0, c0 + CH);
    if constexpr (PER_ROOT) {
      unsigned long long l, hh;
      wave_sum_u128(acc.cnt, &l, &hh);
      if (lane == 0 && (l | hh)) {
        unsigned long long old = atomicAdd(o.per_root + it.r, l);
        if (hh || old + l < old) atomicOr(o.acc + 5, 1ull);
      }
      acc.cnt = 0;
    }
  }
  if constexpr (!PER_ROOT) {
    unsigned long long l, hh;
    wave_sum_u128(acc.cnt, &l, &hh);
    if (lane == 0 && (l | hh)) add_u128(o.acc, l, hh);
  }
}

// ------------------------------------------------------------------ census
//
// Motif census: one persistent launch over (graph, pattern, task) items of
// many graphs and many patterns (k <= 5).  Item t names a (graph, pattern)
// pair through an exclusive prefix over the pairs' task counts, then a
// first-loop task of that pair through the graph's own task prefix; the
// task runs the same loops as k_mine and its count is added to the pair's
// 128-bit accumulator.  The census graphs are small: the loops probe lists
// by binary search only and share the wave pair by pair (no hub bitmaps, no
// whole-wave walks), which keeps the kernels within their registers.

struct CensusPair {
  const int64_t* prefix;  // first-loop task prefix of the pair's graph (n + 1)
  int32_t graph;          // index into the graph table
  int32_t plan;           // index into the plan table
  int32_t chunk;
  int32_t bounded1;
  int32_t out;            // (graph, pattern) slot of the 128-bit accumulators
};

struct CensusArgs {
  const Graph* graphs;
  const Plan* plans;
  const CensusPair* pairs;       // the pairs of one size class
  const long long* pair_prefix;  // n_pairs + 1
  int n_pairs;
  int batch;
  unsigned long long* counts;    // 2 per (graph, pattern) slot
  unsigned long long* queue;     // this class's queue head
};

// one wave's LDS, whatever pattern size its current task has (waves of a
// workgroup may run tasks of different sizes at the same time).  Patterns
// of 2-5 and of 6-7 vertices run in two kernels of the same captured graph,
// so the small ones do not pay the large ones' registers.
template <int KMAX>
union CensusWaveMem;
template <>
union CensusWaveMem<5> {
  WaveMem<2> m2;
  WaveMem<3> m3;
  WaveMem<4> m4;
  WaveMem<5> m5;
};
template <>
union CensusWaveMem<7> {
  WaveMem<6> m6;
  WaveMem<7> m7;
};

template <int K>
__device__ void census_task(const Graph& g, const Plan& plan, WaveMem<K>& M,
                            const CensusPair& pr, long long local, Acc& acc) {
  const int lane = lane_id();
  long long lo = 0, hi = (long long)g.n + 1;
  while (lo < hi) {
    long long mid = (lo + hi) >> 1;
    if (pr.prefix[mid] <= local) lo = mid + 1; else hi = mid;
  }
  const int32_t v0 = uni((int32_t)(lo - 1));
  const int32_t rs0 = uni(g.rowptr[v0]);
  const int32_t rd0 = uni(g.rowptr[v0 + 1]) - rs0;
  const int32_t len1 = pr.bounded1 ? uni(g.lo[v0]) : rd0;
  const int32_t begin = (int32_t)(local - pr.prefix[v0]) * pr.chunk;
  const int32_t end = min(begin + pr.chunk, len1);
  int32_t v[K], rs[K], rd[K];
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = rs[j] = rd[j] = 0;
  v[0] = v0;
  rs[0] = rs0;
  rd[0] = rd0;
  if constexpr (K == 2) {
    if (lane == 0) acc.cnt += (unsigned long long)(end - begin);
  } else if constexpr (K == 3) {
    last_level<K, false, false, false>(g, plan, M, v, rs, rd, 0u, g.col + rs0 + begin, end - begin,
                                       acc);
  } else {
    for (int32_t i = begin; i < end; ++i) {
      v[1] = uni(g.col[rs0 + i]);
      rs[1] = uni(g.rowptr[v[1]]);
      rd[1] = uni(g.rowptr[v[1] + 1]) - rs[1];
      const Split none{nullptr, nullptr, 0, INF, 0};
      mat_level<K, 2, false, false, false>(g, plan, M, v, rs, rd, 0u, acc, none);
    }
  }
}

template <int KMAX>
__global__ __launch_bounds__(BLOCK) void k_census(CensusArgs A) {
  __shared__ CensusWaveMem<KMAX> mem[WPB];
  CensusWaveMem<KMAX>& M = mem[threadIdx.x / WAVE];
  const int lane = lane_id();
  unsigned long long* queue = A.queue;
  const long long n_tasks = A.pair_prefix[A.n_pairs];
  for (;;) {
    long long t0 = 0;
    if (lane == 0) t0 = (long long)atomicAdd(queue, (unsigned long long)A.batch);
    t0 = __shfl(t0, 0, WAVE);
    if (t0 >= n_tasks) break;
    const long long t1 = min(t0 + (long long)A.batch, n_tasks);
    for (long long t = t0; t < t1; ++t) {
      int lo = 0, hi = A.n_pairs + 1;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (A.pair_prefix[mid] <= t) lo = mid + 1; else hi = mid;
      }
      const int pi = lo - 1;
      const CensusPair pr = A.pairs[pi];
      const Graph g = A.graphs[pr.graph];
      const Plan& plan = A.plans[pr.plan];
      const long long local = t - A.pair_prefix[pi];
      Acc acc{0ull, 0ull};
      if constexpr (KMAX == 5) {
        switch (plan.k) {
          case 2: census_task<2>(g, plan, M.m2, pr, local, acc); break;
          case 3: census_task<3>(g, plan, M.m3, pr, local, acc); break;
          case 4: census_task<4>(g, plan, M.m4, pr, local, acc); break;
          default: census_task<5>(g, plan, M.m5, pr, local, acc); break;
        }
      } else {
        if (plan.k == 6) census_task<6>(g, plan, M.m6, pr, local, acc);
        else census_task<7>(g, plan, M.m7, pr, local, acc);
      }
      unsigned long long l, h;
      wave_sum_u128(acc.cnt, &l, &h);
      if (lane == 0 && (l | h)) add_u128(A.counts + 2 * (long long)pr.out, l, h);
    }
  }
}

__global__ void k_fill_u64(unsigned long long* p, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = 0ull;
}

// Test-only preset of the accumulators (GZ_ACC_SEED): the count's low word
// and every per-root slot start at `seed`, so that a small count carries
// into the high word or out of a per-root slot.
__global__ void k_seed_acc(unsigned long long* acc, unsigned long long* per_root, long long n_roots,
                           unsigned long long seed) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) acc[0] = seed;
  for (; i < n_roots; i += (long long)gridDim.x * blockDim.x) per_root[i] = seed;
}

// Neighbour bitmaps of vertices 0..n_hub-1 (rows cleared beforehand): one
// workgroup per hub row at a time, each thread setting the bits of a strided
// share of the hub's neighbours.
__global__ void k_hub_bits(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                           uint32_t* bits, long long row_words, int32_t n_hub) {
  for (int32_t v = blockIdx.x; v < n_hub; v += gridDim.x) {
    uint32_t* row = bits + (long long)v * row_words;
    const int32_t e = rowptr[v + 1];
    for (int32_t i = rowptr[v] + (int32_t)threadIdx.x; i < e; i += (int32_t)blockDim.x) {
      const int32_t x = col[i];
      atomicOr(row + (x >> 5), 1u << (x & 31));
    }
  }
}

}  // namespace dev

// ------------------------------------------------------------ host side

static gz_status upload_prefix(const std::vector<int64_t>& pre, int64_t** out, hipStream_t st);

namespace {

#define GZ_HIP(call)                                                      \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return GZ_EDEVICE;                                                  \
    }                                                                     \
  } while (0)

template <int K, bool PR, bool IN, bool IE>
gz_status launch_k(const dev::Graph& g, const Plan& plan, const dev::Tasks& T,
                   const dev::Out& o, hipStream_t st) {
  auto kern = dev::k_mine<K, PR, IN, IE>;
  int per_cu = 0;
  GZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, dev::BLOCK, 0));
  int devid = 0;
  GZ_HIP(hipGetDevice(&devid));
  int cus = 0;
  GZ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devid));
  long long blocks = (long long)std::max(per_cu, 1) * std::max(cus, 1);
  long long need = (T.n_tasks + (long long)T.batch * dev::WPB - 1) /
                   ((long long)T.batch * dev::WPB);
  blocks = std::max(1ll, std::min(blocks, need));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(dev::BLOCK), 0, st, g, plan, T, o);
  GZ_HIP(hipGetLastError());
  return GZ_OK;
}

template <bool PR, bool IN, bool IE = false>
gz_status launch_by_k(int k, const dev::Graph& g, const Plan& plan,
                      const dev::Tasks& T, const dev::Out& o, hipStream_t st) {
  switch (k) {
    case 2: return launch_k<2, PR, IN, IE>(g, plan, T, o, st);
    case 3: return launch_k<3, PR, IN, IE>(g, plan, T, o, st);
    case 4: return launch_k<4, PR, IN, IE>(g, plan, T, o, st);
    case 5: return launch_k<5, PR, IN, IE>(g, plan, T, o, st);
    case 6: return launch_k<6, PR, IN, IE>(g, plan, T, o, st);
    case 7: return launch_k<7, PR, IN, IE>(g, plan, T, o, st);
    case 8: return launch_k<8, PR, IN, IE>(g, plan, T, o, st);
    default:
      set_error("pattern size out of range");
      return GZ_EINVAL;
  }
}

template <int K, bool PR, int LV>
gz_status launch_heavy_lv(const dev::Graph& g, const Plan& plan, const dev::HeavyItem* items,
                          const long long* prefix, long long n_items, long long n_pieces,
                          unsigned long long* queue, const dev::Out& o, hipStream_t st,
                          bool ie) {
  if constexpr (LV < 2 || LV > K - 2) {
    set_error("split depth outside the materialised loops");
    return GZ_EINVAL;
  } else {
    auto kern = ie ? dev::k_mine_heavy<K, PR, LV, true> : dev::k_mine_heavy<K, PR, LV, false>;
    int per_cu = 0, devid = 0, cus = 0;
    GZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, dev::BLOCK, 0));
    GZ_HIP(hipGetDevice(&devid));
    GZ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devid));
    long long blocks = (long long)std::max(per_cu, 1) * std::max(cus, 1);
    blocks = std::max(1ll, std::min(blocks, (n_pieces + dev::WPB - 1) / dev::WPB));
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(dev::BLOCK), 0, st, g, plan, items,
                       prefix, n_items, queue, o);
    GZ_HIP(hipGetLastError());
    return GZ_OK;
  }
}

template <int K, bool PR>
gz_status launch_heavy_k(int lv, const dev::Graph& g, const Plan& plan,
                         const dev::HeavyItem* items, const long long* prefix, long long n_items,
                         long long n_pieces, unsigned long long* queue, const dev::Out& o,
                         hipStream_t st, bool ie) {
  switch (lv) {
    case 2: return launch_heavy_lv<K, PR, 2>(g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    case 3: return launch_heavy_lv<K, PR, 3>(g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    case 4: return launch_heavy_lv<K, PR, 4>(g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    case 5: return launch_heavy_lv<K, PR, 5>(g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    case 6: return launch_heavy_lv<K, PR, 6>(g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    default:
      set_error("split depth outside the materialised loops");
      return GZ_EINVAL;
  }
}

// An environment variable set to "1".
bool env_flag(const char* name) {
  const char* e = std::getenv(name);
  return e && e[0] == '1' && e[1] == '\0';
}

// GZ_ACC_SEED: a test-only preset of the count accumulators (decimal
// 64-bit value), 0 when unset or malformed.  It shifts every count by the
// seed; tests use it to drive the 128-bit carry and the overflow checks.
unsigned long long acc_seed() {
  const char* e = std::getenv("GZ_ACC_SEED");
  if (!e || !*e || *e == '-') return 0ull;
  char* end = nullptr;
  const unsigned long long v = std::strtoull(e, &end, 10);
  return (end && *end == '\0') ? v : 0ull;
}

// A whole-number environment override within [lo, hi], else `dflt`.
int env_int(const char* name, int dflt, int lo, int hi) {
  const char* e = std::getenv(name);
  if (e && *e) {
    char* end = nullptr;
    const long v = std::strtol(e, &end, 10);
    if (end && *end == '\0' && v >= lo && v <= hi) return (int)v;
  }
  return dflt;
}

// Loop bases longer than this are split (GZ_SPLIT_MIN_LEN overrides).
int split_min_len() {
  const char* e = std::getenv("GZ_SPLIT_MIN_LEN");
  if (e && *e) {
    char* end = nullptr;
    const long v = std::strtol(e, &end, 10);
    if (end && *end == '\0' && v >= 0 && v <= INT32_MAX) return (int)v;
  }
  return 64;
}

// Capacity of the record list (GZ_SPLIT_CAP overrides); prefixes met once
// it is full are expanded in place by the first launch.
long long split_cap() {
  const char* e = std::getenv("GZ_SPLIT_CAP");
  if (e && *e) {
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end && *end == '\0' && v >= 1 && v <= (1ll << 26)) return v;
  }
  return 1ll << 22;
}

// Vertices of at least this degree get a neighbour bitmap (GZ_HUB_MIN_DEG
// overrides, >= 1).
int hub_min_deg() {
  const char* e = std::getenv("GZ_HUB_MIN_DEG");
  if (e && *e) {
    char* end = nullptr;
    const long v = std::strtol(e, &end, 10);
    if (end && *end == '\0' && v >= 1 && v <= INT32_MAX) return (int)v;
  }
  return 512;
}

// Bytes all bitmaps of one graph may take (GZ_HUB_MAX_KB overrides, in KiB;
// 0 switches the bitmaps off).
long long hub_cap_bytes() {
  const char* e = std::getenv("GZ_HUB_MAX_KB");
  if (e && *e) {
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end && *end == '\0' && v >= 0 && v <= (1ll << 40)) return v << 10;
  }
  return 32ll << 30;
}

// The graph's hub bitmaps for the current settings, built on first use and
// kept for the handle's life.  Hubs are the leading run of vertices of
// degree >= hub_min_deg() (after the degree reindex: every such vertex),
// cut to the byte cap.  When the allocation fails the graph simply has no
// hubs: bitmaps only make probes cheaper, never change a result.
gz_status graph_hubs(const gz_graph* g, hipStream_t st, HubMaps* out) {
  const int md = hub_min_deg();
  const long long cap = hub_cap_bytes();
  std::lock_guard<std::mutex> lock(g->task_mu);
  for (const HubMaps& hm : g->hub_cache)
    if (hm.min_deg == md && hm.cap_bytes == cap) {
      *out = hm;
      return GZ_OK;
    }
  const HostGraph& h = g->host;
  HubMaps hm;
  hm.min_deg = md;
  hm.cap_bytes = cap;
  hm.row_words = ((long long)h.n + 31) / 32;
  int32_t H = 0;
  while (H < h.n && h.rowptr[H + 1] - h.rowptr[H] >= md) ++H;
  const long long row_bytes = 4 * hm.row_words;
  if (row_bytes > 0) H = (int32_t)std::min<long long>(H, cap / row_bytes);
  if (H > 0) {
    const long long words = (long long)H * hm.row_words;
    const long long n64 = (words + 1) / 2;
    void* p = nullptr;
    if (hipMalloc(&p, 8 * n64) != hipSuccess) {
      (void)hipGetLastError();
      H = 0;
    } else {
      hipLaunchKernelGGL(dev::k_fill_u64, dim3((unsigned)std::min<long long>((n64 + 255) / 256, 8192)),
                         dim3(256), 0, st, (unsigned long long*)p, n64);
      hipLaunchKernelGGL(dev::k_hub_bits, dim3((unsigned)std::min<int32_t>(H, 8192)), dim3(256), 0,
                         st, g->d_rowptr, g->d_col, (uint32_t*)p, hm.row_words, H);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        (void)hipFree(p);
        set_error(std::string("hub bitmap build: ") + hipGetErrorString(e));
        return GZ_EDEVICE;
      }
      hm.bits = (uint32_t*)p;
    }
  }
  hm.n_hub = H;
  g->hub_cache.push_back(hm);
  *out = hm;
  return GZ_OK;
}

dev::Graph device_graph(const gz_graph* g, const HubMaps& hm) {
  return dev::Graph{g->d_rowptr, g->d_col, g->d_lo, g->host.n, hm.bits, hm.n_hub, hm.row_words};
}

// One launch per loop depth over the recorded prefixes of that depth.
template <bool PR>
gz_status launch_heavy(int k, int lv, const dev::Graph& g, const Plan& plan,
                       const dev::HeavyItem* items, const long long* prefix, long long n_items,
                       long long n_pieces, unsigned long long* queue, const dev::Out& o,
                       hipStream_t st, bool ie) {
  switch (k) {
    case 4: return launch_heavy_k<4, PR>(lv, g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    case 5: return launch_heavy_k<5, PR>(lv, g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    case 6: return launch_heavy_k<6, PR>(lv, g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    case 7: return launch_heavy_k<7, PR>(lv, g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    case 8: return launch_heavy_k<8, PR>(lv, g, plan, items, prefix, n_items, n_pieces, queue, o, st, ie);
    default:
      set_error("split phase needs 4 <= k <= 8");
      return GZ_EINVAL;
  }
}

// Second phase of the generic path: read back the prefixes that phase one
// recorded, group them by loop depth, and hand their bases out in pieces.
gz_status run_heavy(const dev::Graph& dg, const Plan& plan, bool pr, dev::HeavyItem* d_heavy,
                    long long cap, const unsigned long long* d_count, const dev::Out& o,
                    hipStream_t st, void** scratch, bool ie) {
  unsigned long long n_rec = 0;
  hipError_t e = hipMemcpyAsync(&n_rec, d_count, sizeof(n_rec), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const long long n_items = std::min<long long>((long long)n_rec, cap);
  if (e != hipSuccess) {
    set_error(std::string("split list read-back: ") + hipGetErrorString(e));
    return GZ_EDEVICE;
  }
  if (n_items <= 0) return GZ_OK;
  std::vector<dev::HeavyItem> items((size_t)n_items);
  e = hipMemcpy(items.data(), d_heavy, sizeof(dev::HeavyItem) * n_items, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    set_error(std::string("split list read-back: ") + hipGetErrorString(e));
    return GZ_EDEVICE;
  }
  // counting sort by depth; per depth an exclusive prefix over piece counts
  long long cnt[kMaxK + 1] = {0};
  for (const auto& it : items) {
    if (it.level < 2 || it.level > plan.k - 2) {
      set_error("split list holds a record outside the materialised loops");
      return GZ_EDEVICE;
    }
    ++cnt[it.level];
  }
  long long start[kMaxK + 2] = {0};
  for (int lv = 0; lv <= kMaxK; ++lv) start[lv + 1] = start[lv] + cnt[lv];
  std::vector<dev::HeavyItem> sorted((size_t)n_items);
  {
    long long fill[kMaxK + 1];
    for (int lv = 0; lv <= kMaxK; ++lv) fill[lv] = start[lv];
    for (const auto& it : items) sorted[(size_t)fill[it.level]++] = it;
  }
  // prefix of depth lv at offset start[lv] + lv (one extra entry per depth)
  std::vector<long long> pre((size_t)n_items + kMaxK + 1, 0);
  long long pieces[kMaxK + 1] = {0};
  for (int lv = 2; lv <= plan.k - 2; ++lv) {
    const long long off = start[lv] + lv;
    pre[(size_t)off] = 0;
    for (long long i = 0; i < cnt[lv]; ++i)
      pre[(size_t)(off + i + 1)] =
          pre[(size_t)(off + i)] + (sorted[(size_t)(start[lv] + i)].base_len + dev::CH - 1) / dev::CH;
    pieces[lv] = pre[(size_t)(off + cnt[lv])];
  }
  char* buf = nullptr;
  const size_t q_bytes = 256;
  const size_t p_bytes = sizeof(long long) * pre.size();
  if (hipMalloc(&buf, q_bytes + p_bytes) != hipSuccess) {
    set_error("device allocation of the split prefix failed");
    return GZ_ENOMEM;
  }
  *scratch = buf;
  unsigned long long* queues = (unsigned long long*)buf;
  long long* d_pre = (long long*)(buf + q_bytes);
  if (hipMemcpy(d_heavy, sorted.data(), sizeof(dev::HeavyItem) * n_items,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_pre, pre.data(), p_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    set_error("split prefix upload failed");
    return GZ_EDEVICE;
  }
  hipLaunchKernelGGL(dev::k_fill_u64, dim3(1), dim3(256), 0, st, queues, (long long)(kMaxK + 1));
  for (int lv = 2; lv <= plan.k - 2; ++lv) {
    if (!cnt[lv]) continue;
    gz_status rc = pr ? launch_heavy<true>(plan.k, lv, dg, plan, d_heavy + start[lv],
                                           d_pre + start[lv] + lv, cnt[lv], pieces[lv],
                                           queues + lv, o, st, ie)
                      : launch_heavy<false>(plan.k, lv, dg, plan, d_heavy + start[lv],
                                            d_pre + start[lv] + lv, cnt[lv], pieces[lv],
                                            queues + lv, o, st, ie);
    if (rc) return rc;
  }
  return GZ_OK;
}

int chunk_for(int k) { return k <= 2 ? (1 << 30) : (k == 3 ? 64 : 16); }

// K_k with every loop bounded by the previous one
bool is_clique_chain(const Plan& p) {
  for (int i = 1; i < p.k; ++i)
    if (p.lv[i].isect != (uint8_t)((1u << i) - 1) || p.lv[i].sub != 0 || p.lv[i].bound != i - 1)
      return false;
  return true;
}

gz_status upload_i32(const std::vector<int32_t>& v, int32_t** out, hipStream_t st) {
  *out = nullptr;
  if (v.empty()) return GZ_OK;
  GZ_HIP(hipMalloc(out, v.size() * sizeof(int32_t)));
  GZ_HIP(hipMemcpyAsync(*out, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  return GZ_OK;
}

gz_status build_clique_lists(const HostGraph& h, const int32_t* roots, int64_t n_roots,
                             int32_t max_lo, int32_t chunk, hipStream_t st, CliqueLists* out) {
  std::vector<int32_t> lv, lr, ov, orr;
  std::vector<int64_t> opre(1, 0);
  std::vector<std::pair<int32_t, int32_t>> hv;  // (lo, index)
  const int64_t nr = roots ? n_roots : h.n;
  out->max_lo = max_lo;
  for (int64_t i = 0; i < nr; ++i) {
    const int32_t v = roots ? roots[i] : (int32_t)i;
    const int32_t d = h.lo[v];
    if (d < 3) continue;
    if (d > max_lo) {
      ov.push_back(v);
      orr.push_back((int32_t)i);
      opre.push_back(opre.back() + (d + chunk - 1) / chunk);
    } else if (d <= dev::CW) {
      lv.push_back(v);
      lr.push_back((int32_t)i);
    } else {
      hv.emplace_back(d, (int32_t)i);
    }
  }
  std::stable_sort(hv.begin(), hv.end(),
                   [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
                     return a.first > b.first;
                   });
  std::vector<int32_t> hvv, hvr;
  // size classes of 2, 4 and 8 words, then the rest: smaller rows take less
  // LDS, so more workgroups share a CU
  const int32_t classes[3] = {2, 4, 8};
  out->n_buckets = 0;
  for (size_t i = 0; i < hv.size(); ++i) {
    const auto& x = hv[i];
    hvv.push_back(roots ? roots[x.second] : x.second);
    hvr.push_back(x.second);
    out->heavy_max_lo = std::max(out->heavy_max_lo, x.first);
  }
  {
    // walk from the smallest roots (the end) up, closing a class when the
    // next root needs more words
    const int64_t nh = (int64_t)hv.size();
    int32_t ws[4];
    int64_t ends[4];
    int nb = 0;
    int64_t i = nh;
    for (int c = 0; c < 3 && i > 0; ++c) {
      int64_t j = i;
      while (j > 0 && (hv[(size_t)(j - 1)].first + 63) / 64 <= classes[c]) --j;
      if (j < i) {
        ws[nb] = classes[c];
        ends[nb] = i;
        ++nb;
        i = j;
      }
    }
    if (i > 0) {
      ws[nb] = (hv[0].first + 63) / 64;
      ends[nb] = i;
      ++nb;
    }
    // classes from the largest rows (front of the list) to the smallest
    int64_t begin = 0;
    for (int b = 0; b < nb; ++b) {
      const int src = nb - 1 - b;
      out->bucket_w[b] = ws[src];
      out->bucket_begin[b] = begin;
      begin = ends[src];
    }
    out->bucket_begin[nb] = begin;
    out->n_buckets = nb;
  }
  gz_status rc = upload_i32(lv, &out->light_v, st);
  if (!rc) rc = upload_i32(lr, &out->light_r, st);
  if (!rc) rc = upload_i32(hvv, &out->heavy_v, st);
  if (!rc) rc = upload_i32(hvr, &out->heavy_r, st);
  if (!rc && !ov.empty()) {
    rc = upload_i32(ov, &out->over_v, st);
    if (!rc) rc = upload_i32(orr, &out->over_r, st);
    if (!rc) rc = upload_prefix(opre, &out->over_prefix, st);
  }
  if (!rc && hipStreamSynchronize(st) != hipSuccess) {
    set_error("clique root list upload failed");
    rc = GZ_EDEVICE;
  }
  out->n_light = (int64_t)lv.size();
  out->n_heavy = (int64_t)hvv.size();
  out->n_over = (int64_t)ov.size();
  out->over_tasks = opre.back();
  return rc;
}

void free_clique_lists(CliqueLists* c) {
  for (int32_t* p : {c->light_v, c->light_r, c->heavy_v, c->heavy_r, c->over_v, c->over_r})
    if (p) (void)hipFree(p);
  if (c->over_prefix) (void)hipFree(c->over_prefix);
  *c = CliqueLists();
}

// Side streams of the current device (default priority, created once, kept
// for the process): the clique size classes run on them concurrently.
hipStream_t side_stream(int i) {
  static std::mutex mu;
  static hipStream_t streams[16][4] = {};
  int dev_id = 0;
  if (hipGetDevice(&dev_id) != hipSuccess || dev_id < 0 || dev_id >= 16 || i < 0 || i >= 4)
    return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev_id][i] &&
      hipStreamCreateWithFlags(&streams[dev_id][i], hipStreamNonBlocking) != hipSuccess)
    streams[dev_id][i] = nullptr;
  return streams[dev_id][i];
}

template <int K, bool PR, bool IN>
gz_status launch_clique_k(const dev::Graph& g, const CliqueLists& C, const dev::Out& o,
                          hipStream_t st) {
  int devid = 0, cus = 0, per_cu = 0;
  GZ_HIP(hipGetDevice(&devid));
  GZ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devid));
  // the size classes below start with the wave path, not after it
  hipEvent_t fork = nullptr;
  if (C.n_buckets > 0 && (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
                          hipEventRecord(fork, st) != hipSuccess)) {
    if (fork) (void)hipEventDestroy(fork);
    set_error("clique fork event failed");
    return GZ_EDEVICE;
  }
  if (C.n_light > 0) {
    const int batch = 8;
    auto kw = dev::k_clique_wave<K, PR, IN>;
    GZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kw, dev::BLOCK, 0));
    long long blocks = (long long)std::max(per_cu, 1) * std::max(cus, 1);
    long long need = (C.n_light + (long long)batch * dev::WPB - 1) / ((long long)batch * dev::WPB);
    blocks = std::max(1ll, std::min(blocks, need));
    dev::RootList L{C.light_v, C.light_r, C.n_light};
    hipLaunchKernelGGL(kw, dim3((unsigned)blocks), dim3(dev::BLOCK), 0, st, g, L, o, batch);
    if (hipGetLastError() != hipSuccess) {
      if (fork) (void)hipEventDestroy(fork);
      set_error("clique wave launch failed");
      return GZ_EDEVICE;
    }
  }
  // one launch per size class, each with its own queue, on side streams so
  // that the classes share the CUs instead of each draining alone
  if (C.n_buckets <= 0) return GZ_OK;
  hipStream_t side[4];
  hipEvent_t join[4] = {nullptr, nullptr, nullptr, nullptr};
  gz_status rc = GZ_OK;
  for (int b = 0; b < C.n_buckets && !rc; ++b) {
    side[b] = side_stream(b);
    if (!side[b]) {
      set_error("side stream creation failed");
      rc = GZ_EDEVICE;
    }
  }
  for (int b = 0; b < C.n_buckets && !rc; ++b) {
    const long long n_b = C.bucket_begin[b + 1] - C.bucket_begin[b];
    auto kb = dev::k_clique_block<K, PR, IN>;
    const int W = C.bucket_w[b];
    const size_t S = 64 * (size_t)W;
    const size_t lds = S * W * sizeof(unsigned long long) + 5 * S * sizeof(int32_t) +
                       dev::FILT_WORDS * sizeof(uint32_t);
    if (hipFuncSetAttribute((const void*)kb, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kb, dev::CBLOCK, lds) !=
            hipSuccess ||
        per_cu < 1) {
      set_error("clique workgroup path does not fit in LDS");
      rc = GZ_EDEVICE;
      break;
    }
    if (hipStreamWaitEvent(side[b], fork, 0) != hipSuccess ||
        hipEventCreateWithFlags(&join[b], hipEventDisableTiming) != hipSuccess) {
      set_error("clique stream fork failed");
      rc = GZ_EDEVICE;
      break;
    }
    long long blocks = std::min<long long>((long long)per_cu * std::max(cus, 1), n_b);
    dev::RootList L{C.heavy_v + C.bucket_begin[b], C.heavy_r + C.bucket_begin[b], n_b};
    hipLaunchKernelGGL(kb, dim3((unsigned)std::max(blocks, 1ll)), dim3(dev::CBLOCK), lds, side[b],
                       g, L, o, W, o.acc + dev::ACC_BLOCK_QUEUES + b);
    if (hipGetLastError() != hipSuccess || hipEventRecord(join[b], side[b]) != hipSuccess ||
        hipStreamWaitEvent(st, join[b], 0) != hipSuccess) {
      set_error("clique workgroup launch failed");
      rc = GZ_EDEVICE;
      break;
    }
  }
  if (fork) (void)hipEventDestroy(fork);
  for (hipEvent_t e : join)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

template <bool PR, bool IN>
gz_status launch_clique(int k, const dev::Graph& g, const CliqueLists& C, const dev::Out& o,
                        hipStream_t st) {
  switch (k) {
    case 4: return launch_clique_k<4, PR, IN>(g, C, o, st);
    case 5: return launch_clique_k<5, PR, IN>(g, C, o, st);
    case 6: return launch_clique_k<6, PR, IN>(g, C, o, st);
    case 7: return launch_clique_k<7, PR, IN>(g, C, o, st);
    case 8: return launch_clique_k<8, PR, IN>(g, C, o, st);
    default:
      set_error("clique path needs 4 <= k <= 8");
      return GZ_EINVAL;
  }
}

}  // namespace

// First-loop length of a root, for the task split.
static inline int64_t len1_of(const HostGraph& h, int32_t v, bool bounded1) {
  return bounded1 ? h.lo[v] : (h.rowptr[v + 1] - h.rowptr[v]);
}

static gz_status upload_prefix(const std::vector<int64_t>& pre, int64_t** out,
                               hipStream_t st) {
  int64_t* d = nullptr;
  GZ_HIP(hipMalloc(&d, pre.size() * sizeof(int64_t)));
  hipError_t e = hipMemcpyAsync(d, pre.data(), pre.size() * sizeof(int64_t),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipFree(d);
    set_error(std::string("task prefix upload: ") + hipGetErrorString(e));
    return GZ_EDEVICE;
  }
  *out = d;
  return GZ_OK;
}

// Cached all-roots task prefix for (bounded1, chunk).
static gz_status graph_tasks(const gz_graph* g, bool bounded1, int chunk,
                             hipStream_t st, DevTasks* out) {
  const int64_t key = (int64_t)chunk * 2 + (bounded1 ? 1 : 0);
  std::lock_guard<std::mutex> lock(g->task_mu);
  for (auto& kv : g->task_cache)
    if (kv.first == key) {
      *out = kv.second;
      return GZ_OK;
    }
  const HostGraph& h = g->host;
  std::vector<int64_t> pre((size_t)h.n + 1, 0);
  for (int32_t v = 0; v < h.n; ++v)
    pre[v + 1] = pre[v] + (len1_of(h, v, bounded1) + chunk - 1) / chunk;
  DevTasks dt;
  dt.n_tasks = pre[h.n];
  gz_status rc = upload_prefix(pre, &dt.prefix, st);
  if (rc) return rc;
  g->task_cache.emplace_back(key, dt);
  *out = dt;
  return GZ_OK;
}

// Task lists of the first loop for every (bounded, chunk) a generic count
// can ask for (chunks of 16 and 64 candidates), built when the graph is
// loaded so that gz_count_noalloc finds them.
gz_status prepare_graph_tasks(const gz_graph* g, hipStream_t st) {
  for (int b = 0; b < 2; ++b)
    for (int chunk : {16, 64}) {
      DevTasks t;
      gz_status rc = graph_tasks(g, b != 0, chunk, st, &t);
      if (rc) return rc;
    }
  return GZ_OK;
}

// ---------------------------------------------------- allocation-free count
//
// gz_count_noalloc keeps its accumulators (the 128-bit count, the queue head
// and the rest of the layout of k_mine's acc) in this file-scope device
// array instead of a per-call allocation.  Each GPU holds its own copy at
// its own address until the process ends; host code must use that address
// (looked up once per device below), never the array's name.  Every call on
// a GPU shares the array and clears it first: calls that overlap on one GPU
// race.
constexpr int NOALLOC_ACC_WORDS = dev::ACC_HEAD;
__device__ __align__(256) unsigned long long scratch[NOALLOC_ACC_WORDS];

static gz_status scratch_address(unsigned long long** out) {
  static std::mutex mu;
  static unsigned long long* addr[64] = {};
  int devid = 0;
  GZ_HIP(hipGetDevice(&devid));
  if (devid < 0 || devid >= 64) {
    set_error("device index out of range for the scratch table");
    return GZ_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[devid]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("scratch address: ") + hipGetErrorString(e));
      return GZ_EDEVICE;
    }
    addr[devid] = (unsigned long long*)ptr;
  }
  *out = addr[devid];
  return GZ_OK;
}

// The last loop's evaluation choices of a count call, from the environment
// (defaults otherwise); none of them changes a result.
void plan_knobs(Plan& plan) {
  plan.ie_force = env_flag("GZ_IE_FORCE");
  plan.long_min = env_int("GZ_LONG_MIN", 256, 1, 1 << 30);
  plan.merge_ratio = env_int("GZ_MERGE_RATIO", 4, 0, 1 << 20);
  plan.ie_ratio = env_int("GZ_IE_RATIO", 12, 0, 1 << 20);
  plan.sweep_min = env_int("GZ_SWEEP_MIN", 16384, 0, INT32_MAX);
  plan.sweep_ie = env_int("GZ_SWEEP_IE", 2, 0, 1 << 20);
}

// gz_count without any device allocation: the generic kernels over every
// root with the graph's task list from load time, the hub bitmaps only if a
// count has already built them, and no two-phase split (its record list is
// per call): long loop bases are expanded by the wave that meets them.
gz_status run_count_noalloc(const gz_graph* g, const gz_schedule* s, hipStream_t st,
                            unsigned __int128* total) {
  Plan plan = s->plan;
  plan_knobs(plan);
  const HostGraph& h = g->host;
  const bool bounded1 = plan.lv[1].bound == 0;
  const int chunk = plan.k == 3 ? 64 : 16;
  DevTasks tasks;
  bool have = false;
  HubMaps hubs;
  {
    std::lock_guard<std::mutex> lock(g->task_mu);
    const int64_t key = (int64_t)chunk * 2 + (bounded1 ? 1 : 0);
    for (auto& kv : g->task_cache)
      if (kv.first == key) {
        tasks = kv.second;
        have = true;
      }
    for (const HubMaps& hm : g->hub_cache)
      if (hm.min_deg == hub_min_deg() && hm.cap_bytes == hub_cap_bytes()) hubs = hm;
  }
  if (!have) {
    set_error("the graph has no first-loop task list (it is built when the graph is loaded)");
    return GZ_ENOTSUP;
  }
  unsigned long long* acc = nullptr;
  gz_status rc = scratch_address(&acc);
  if (rc) return rc;
  const bool ie = plan.k >= 3 && plan.lv[plan.k - 1].sub != 0;
  hipLaunchKernelGGL(dev::k_fill_u64, dim3(1), dim3(64), 0, st, acc, (long long)NOALLOC_ACC_WORDS);
  GZ_HIP(hipGetLastError());
  if (tasks.n_tasks > 0) {
    const dev::Graph dg = device_graph(g, hubs);
    dev::Tasks dt{tasks.prefix, nullptr, nullptr, h.n, tasks.n_tasks, chunk, bounded1 ? 1 : 0, 1,
                  INT32_MAX, nullptr, 0, 4};
    dev::Out o{acc, nullptr};
    rc = ie ? launch_by_k<false, false, true>(plan.k, dg, plan, dt, o, st)
            : launch_by_k<false, false>(plan.k, dg, plan, dt, o, st);
    if (rc) return rc;
  }
  unsigned long long res[2] = {0ull, 0ull};
  hipError_t e = hipMemcpyAsync(res, acc, sizeof(res), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_error(std::string("mining kernel: ") + hipGetErrorString(e));
    return GZ_EDEVICE;
  }
  *total = ((unsigned __int128)res[1] << 64) | res[0];
  return GZ_OK;
}

gz_status run_count(const gz_graph* g, const gz_schedule* s, hipStream_t st,
                    const int32_t* roots, int64_t n_roots, uint64_t* per_root,
                    bool instr, unsigned __int128* total, unsigned __int128* bytes,
                    float* kernel_ms, bool clique_ops) {
  Plan plan = s->plan;
  plan_knobs(plan);
  const HostGraph& h = g->host;
  const bool bounded1 = plan.lv[1].bound == 0;
  const int chunk = chunk_for(plan.k);
  const bool pr = roots != nullptr;         // a root list is given
  const bool out_pr = per_root != nullptr;  // per-root counts are wanted

  DevTasks tasks;
  int64_t* own_prefix = nullptr;
  int32_t* d_roots = nullptr;
  int64_t nr = h.n;
  if (!pr) {
    gz_status rc = graph_tasks(g, bounded1, chunk, st, &tasks);
    if (rc) return rc;
  } else {
    nr = n_roots;
    std::vector<int64_t> pre((size_t)nr + 1, 0);
    for (int64_t i = 0; i < nr; ++i)
      pre[i + 1] = pre[i] + (len1_of(h, roots[i], bounded1) + chunk - 1) / chunk;
    tasks.n_tasks = pre[nr];
    gz_status rc = upload_prefix(pre, &own_prefix, st);
    if (rc) return rc;
    tasks.prefix = own_prefix;
    if (hipMalloc(&d_roots, sizeof(int32_t) * std::max<int64_t>(nr, 1)) != hipSuccess ||
        hipMemcpyAsync(d_roots, roots, sizeof(int32_t) * nr, hipMemcpyHostToDevice, st) !=
            hipSuccess) {
      (void)hipFree(own_prefix);
      (void)hipFree(d_roots);
      set_error("root list upload failed");
      return GZ_EDEVICE;
    }
  }

  unsigned long long* d_acc = nullptr;
  const long long n_acc = dev::ACC_HEAD + (out_pr ? nr : 0);
  gz_status rc = GZ_OK;
  if (hipMalloc(&d_acc, sizeof(unsigned long long) * n_acc) != hipSuccess) {
    set_error("device allocation of the accumulators failed");
    rc = GZ_ENOMEM;
  }
  // clique fast path: K_k (k >= 4) with chain bounds; roots with more
  // candidates than the bit rows hold (GZ_CLIQUE_MAX_LO, at most 1024)
  // take the generic loops through a root list
  const bool use_clique = !instr && plan.k >= 4 && is_clique_chain(plan);
  const int32_t clique_max_lo = env_int("GZ_CLIQUE_MAX_LO", 1024, 0, 1024);
  CliqueLists own_lists;
  const CliqueLists* lists = nullptr;
  if (!rc && use_clique) {
    if (!pr && clique_max_lo == 1024) {
      std::lock_guard<std::mutex> lock(g->task_mu);
      if (!g->clique_ready) {
        rc = build_clique_lists(h, nullptr, 0, 1024, 1, st, &g->clique_all);
        if (rc) free_clique_lists(&g->clique_all);
        else g->clique_ready = true;
      }
      lists = &g->clique_all;
    } else {
      rc = build_clique_lists(h, roots, nr, clique_max_lo, 1, st, &own_lists);
      lists = &own_lists;
    }
  }
  const bool over = use_clique && lists && lists->n_over > 0;
  if (!rc && clique_ops && (!use_clique || pr || over)) {
    set_error("operation counts exist only for the clique path over all roots");
    rc = GZ_ENOTSUP;
  }
  // inclusion-exclusion in the last loop: wherever it has negative lists
  const bool ie = !instr && plan.k >= 3 && plan.lv[plan.k - 1].sub != 0;
  // second phase of the generic path: long loop bases split into pieces
  const bool split = !rc && (!use_clique || over) && !instr && plan.k >= 4;
  const long long heavy_cap = split ? split_cap() : 0;
  dev::HeavyItem* d_heavy = nullptr;
  if (split && hipMalloc(&d_heavy, sizeof(dev::HeavyItem) * heavy_cap) != hipSuccess) {
    set_error("device allocation of the split list failed");
    rc = GZ_ENOMEM;
  }
  // neighbour bitmaps of the hubs for the generic path's probes
  HubMaps hubs;
  if (!rc && (!use_clique || over)) rc = graph_hubs(g, st, &hubs);
  void* heavy_scratch = nullptr;
  if (!rc) {
    hipLaunchKernelGGL(dev::k_fill_u64, dim3((unsigned)std::min<long long>((n_acc + 255) / 256, 4096)),
                       dim3(256), 0, st, d_acc, n_acc);
    if (const unsigned long long seed = acc_seed())
      hipLaunchKernelGGL(dev::k_seed_acc, dim3((unsigned)std::min<long long>((nr + 255) / 256 + 1, 4096)),
                         dim3(256), 0, st, d_acc, d_acc + dev::ACC_HEAD, out_pr ? nr : 0ll, seed);
    const dev::Graph dg = device_graph(g, hubs);
    dev::Tasks dt{tasks.prefix, d_roots, nullptr, nr, tasks.n_tasks, chunk, bounded1 ? 1 : 0, 1,
                  split_min_len(), d_heavy, split ? heavy_cap : 0, 4};
    dev::Out o{d_acc, d_acc + dev::ACC_HEAD};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (kernel_ms) {
      *kernel_ms = 0.0f;
      if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess ||
          hipEventRecord(ev0, st) != hipSuccess) {
        set_error("hipEvent set-up failed");
        rc = GZ_EDEVICE;
      }
    }
    if (!rc && tasks.n_tasks > 0) {
      if (use_clique) {
        rc = out_pr ? launch_clique<true, false>(plan.k, dg, *lists, o, st)
                : (clique_ops ? launch_clique<false, true>(plan.k, dg, *lists, o, st)
                              : launch_clique<false, false>(plan.k, dg, *lists, o, st));
        if (!rc && over) {
          // few roots with dense candidate sets: one first-loop candidate
          // per task and every base longer than a piece split
          const dev::Tasks ot{lists->over_prefix, lists->over_v, lists->over_r, lists->n_over,
                              lists->over_tasks, 1, 1, 1, std::min(split_min_len(), dev::CH),
                              d_heavy, heavy_cap, 7};
          rc = out_pr ? launch_by_k<true, false>(plan.k, dg, plan, ot, o, st)
                      : launch_by_k<false, false>(plan.k, dg, plan, ot, o, st);
        }
      } else if (out_pr && instr) rc = launch_by_k<true, true>(plan.k, dg, plan, dt, o, st);
      else if (out_pr) rc = ie ? launch_by_k<true, false, true>(plan.k, dg, plan, dt, o, st)
                           : launch_by_k<true, false>(plan.k, dg, plan, dt, o, st);
      else if (instr) rc = launch_by_k<false, true>(plan.k, dg, plan, dt, o, st);
      else rc = ie ? launch_by_k<false, false, true>(plan.k, dg, plan, dt, o, st)
                   : launch_by_k<false, false>(plan.k, dg, plan, dt, o, st);
    }
    if (!rc && split && tasks.n_tasks > 0)
      rc = run_heavy(dg, plan, out_pr, d_heavy, heavy_cap, d_acc + 6, o, st, &heavy_scratch, ie);
    if (kernel_ms && !rc) {
      if (hipEventRecord(ev1, st) != hipSuccess || hipEventSynchronize(ev1) != hipSuccess ||
          hipEventElapsedTime(kernel_ms, ev0, ev1) != hipSuccess) {
        set_error("hipEvent timing failed");
        rc = GZ_EDEVICE;
      }
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
  std::vector<unsigned long long> hacc((size_t)n_acc, 0ull);
  if (!rc) {
    hipError_t e = hipMemcpyAsync(hacc.data(), d_acc, sizeof(unsigned long long) * n_acc,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      set_error(std::string("mining kernel: ") + hipGetErrorString(e));
      rc = GZ_EDEVICE;
    }
  }
  (void)hipFree(d_acc);
  if (d_heavy) (void)hipFree(d_heavy);
  if (heavy_scratch) (void)hipFree(heavy_scratch);
  free_clique_lists(&own_lists);
  if (own_prefix) (void)hipFree(own_prefix);
  if (d_roots) (void)hipFree(d_roots);
  if (rc) return rc;

  *total = ((unsigned __int128)hacc[1] << 64) | hacc[0];
  if (bytes && clique_ops) {
    *bytes = ((unsigned __int128)hacc[3] << 64) | hacc[2];
  } else if (bytes) {
    unsigned __int128 b = ((unsigned __int128)hacc[3] << 64) | hacc[2];
    // loop 1 is evaluated once per root: one list, N(v0), below its bound
    for (int64_t i = 0; i < nr; ++i) {
      int32_t v0 = pr ? roots[i] : (int32_t)i;
      b += (unsigned __int128)(4 * len1_of(h, v0, bounded1) + 8);
    }
    *bytes = b;
  }
  if (out_pr) {
    if (hacc[5]) {
      set_error("a per-root count does not fit in 64 bits");
      return GZ_EOVERFLOW;
    }
    for (int64_t i = 0; i < nr; ++i) per_root[i] = hacc[dev::ACC_HEAD + i];
  }
  return GZ_OK;
}


// ------------------------------------------------------------ census host

void census_free(void* p);

struct gz_census_impl {
  std::vector<const gz_graph*> graphs;
  std::vector<const gz_schedule*> scheds;
  int device = 0;
  hipStream_t stream = nullptr;
  dev::Graph* d_graphs = nullptr;
  Plan* d_plans = nullptr;
  // per size class (patterns of 2-5 and of 6-7 vertices): pair table,
  // task prefix and launch size
  dev::CensusPair* d_pairs[2] = {nullptr, nullptr};
  long long* d_pair_prefix[2] = {nullptr, nullptr};
  int n_class_pairs[2] = {0, 0};
  long long class_tasks[2] = {0, 0};
  int class_grid[2] = {0, 0};
  unsigned long long* d_counts = nullptr;  // 2 per pair, then 2 queue heads
  int n_pairs = 0;
  long long n_tasks = 0;
  // defaults: the tuner's pick on the smallest graphs of the 64-graph batch
  int chunk3 = 128, chunk45 = 1, batch = 1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void census_release_tables(gz_census_impl* c) {
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->exec = nullptr;
  c->graph = nullptr;
  for (int k = 0; k < 2; ++k) {
    if (c->d_pairs[k]) (void)hipFree(c->d_pairs[k]);
    if (c->d_pair_prefix[k]) (void)hipFree(c->d_pair_prefix[k]);
    c->d_pairs[k] = nullptr;
    c->d_pair_prefix[k] = nullptr;
  }
}

// Pair table and prefix for the current tuning, then capture the zeroing of
// the accumulators and the census launch into a HIP graph.
static gz_status census_build(gz_census_impl* c) {
  census_release_tables(c);
  const int ng = (int)c->graphs.size(), ns = (int)c->scheds.size();
  std::vector<dev::CensusPair> pairs[2];
  std::vector<long long> prefix[2] = {{0}, {0}};
  for (int gi = 0; gi < ng; ++gi)
    for (int si = 0; si < ns; ++si) {
      const Plan& pl = c->scheds[si]->plan;
      const bool b1 = pl.lv[1].bound == 0;
      const int chunk = pl.k <= 2 ? (1 << 30) : (pl.k == 3 ? c->chunk3 : c->chunk45);
      DevTasks dt;
      gz_status rc = graph_tasks(c->graphs[gi], b1, chunk, c->stream, &dt);
      if (rc) return rc;
      const int cls = pl.k <= 5 ? 0 : 1;
      pairs[cls].push_back(dev::CensusPair{dt.prefix, gi, si, chunk, b1 ? 1 : 0, gi * ns + si});
      prefix[cls].push_back(prefix[cls].back() + dt.n_tasks);
    }
  c->n_pairs = ng * ns;
  c->n_tasks = prefix[0].back() + prefix[1].back();
  int cus = 0;
  GZ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  for (int cls = 0; cls < 2; ++cls) {
    c->n_class_pairs[cls] = (int)pairs[cls].size();
    c->class_tasks[cls] = prefix[cls].back();
    if (pairs[cls].empty()) continue;
    GZ_HIP(hipMalloc(&c->d_pairs[cls], sizeof(dev::CensusPair) * pairs[cls].size()));
    GZ_HIP(hipMalloc(&c->d_pair_prefix[cls], sizeof(long long) * prefix[cls].size()));
    GZ_HIP(hipMemcpy(c->d_pairs[cls], pairs[cls].data(),
                     sizeof(dev::CensusPair) * pairs[cls].size(), hipMemcpyHostToDevice));
    GZ_HIP(hipMemcpy(c->d_pair_prefix[cls], prefix[cls].data(),
                     sizeof(long long) * prefix[cls].size(), hipMemcpyHostToDevice));
    int per_cu = 0;
    if (cls == 0)
      GZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dev::k_census<5>, dev::BLOCK, 0));
    else
      GZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dev::k_census<7>, dev::BLOCK, 0));
    const long long need = (c->class_tasks[cls] + (long long)c->batch * dev::WPB - 1) /
                           ((long long)c->batch * dev::WPB);
    c->class_grid[cls] =
        (int)std::max(1ll, std::min((long long)std::max(per_cu, 1) * std::max(cus, 1), need));
  }
  const long long n_acc = 2LL * c->n_pairs + 2;
  unsigned long long* queues = c->d_counts + 2LL * c->n_pairs;
  GZ_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(dev::k_fill_u64, dim3((unsigned)std::min<long long>((n_acc + 255) / 256, 4096)),
                     dim3(256), 0, c->stream, c->d_counts, n_acc);
  for (int cls = 0; cls < 2; ++cls) {
    if (c->class_tasks[cls] <= 0) continue;
    dev::CensusArgs args{c->d_graphs, c->d_plans, c->d_pairs[cls], c->d_pair_prefix[cls],
                         c->n_class_pairs[cls], c->batch, c->d_counts, queues + cls};
    if (cls == 0)
      hipLaunchKernelGGL(dev::k_census<5>, dim3((unsigned)c->class_grid[cls]), dim3(dev::BLOCK), 0,
                         c->stream, args);
    else
      hipLaunchKernelGGL(dev::k_census<7>, dim3((unsigned)c->class_grid[cls]), dim3(dev::BLOCK), 0,
                         c->stream, args);
  }
  hipError_t e = hipStreamEndCapture(c->stream, &c->graph);
  if (e != hipSuccess) {
    set_error(std::string("census graph capture: ") + hipGetErrorString(e));
    return GZ_EDEVICE;
  }
  GZ_HIP(hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
  return GZ_OK;
}

static gz_status census_launch(gz_census_impl* c, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GZ_HIP(hipEventCreate(&e0));
  GZ_HIP(hipEventCreate(&e1));
  gz_status rc = GZ_OK;
  if (hipEventRecord(e0, c->stream) != hipSuccess || hipGraphLaunch(c->exec, c->stream) != hipSuccess ||
      hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(ms, e0, e1) != hipSuccess) {
    set_error("census launch failed");
    rc = GZ_EDEVICE;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

gz_status census_create(const gz_graph* const* graphs, int32_t n_graphs,
                        const gz_schedule* const* scheds, int32_t n_scheds, void** out) {
  if (!out || n_graphs < 1 || n_scheds < 1 || !graphs || !scheds) {
    set_error("bad census arguments");
    return GZ_EINVAL;
  }
  auto* c = new (std::nothrow) gz_census_impl();
  if (!c) {
    set_error("out of host memory");
    return GZ_ENOMEM;
  }
  gz_status rc = GZ_OK;
  if (hipGetDevice(&c->device) != hipSuccess) rc = GZ_EDEVICE;
  for (int i = 0; i < n_graphs && !rc; ++i) {
    if (!graphs[i] || graphs[i]->device != c->device) {
      set_error("census graphs must be loaded on the current device");
      rc = GZ_EINVAL;
    }
  }
  for (int i = 0; i < n_scheds && !rc; ++i) {
    if (!scheds[i] || scheds[i]->plan.k > 7) {
      set_error("census patterns must have at most 7 vertices");
      rc = scheds[i] ? GZ_ENOTSUP : GZ_EINVAL;
    }
  }
  if (!rc) {
    c->graphs.assign(graphs, graphs + n_graphs);
    c->scheds.assign(scheds, scheds + n_scheds);
  }
  std::vector<dev::Graph> gt;
  for (int i = 0; i < n_graphs && !rc; ++i) gt.push_back(device_graph(graphs[i], HubMaps{}));
  if (!rc) {
    std::vector<Plan> pt;
    for (const gz_schedule* s : c->scheds) pt.push_back(s->plan);
    if (hipStreamCreate(&c->stream) != hipSuccess ||
        hipMalloc(&c->d_graphs, sizeof(dev::Graph) * gt.size()) != hipSuccess ||
        hipMalloc(&c->d_plans, sizeof(Plan) * pt.size()) != hipSuccess ||
        hipMalloc(&c->d_counts, sizeof(unsigned long long) * (2 * (size_t)n_graphs * n_scheds + 2)) !=
            hipSuccess ||
        hipMemcpy(c->d_graphs, gt.data(), sizeof(dev::Graph) * gt.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_plans, pt.data(), sizeof(Plan) * pt.size(), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("census device set-up failed");
      rc = GZ_EDEVICE;
    }
  }
  if (!rc) rc = census_build(c);
  if (rc) {
    census_free(c);
    return rc;
  }
  *out = c;
  return GZ_OK;
}

void census_free(void* p) {
  auto* c = (gz_census_impl*)p;
  if (!c) return;
  census_release_tables(c);
  for (void* q : {(void*)c->d_graphs, (void*)c->d_plans, (void*)c->d_counts})
    if (q) (void)hipFree(q);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

gz_status census_run(void* p, uint64_t* counts, float* ms) {
  auto* c = (gz_census_impl*)p;
  float t = 0.0f;
  gz_status rc = census_launch(c, &t);
  if (rc) return rc;
  std::vector<unsigned long long> h(2 * (size_t)c->n_pairs);
  GZ_HIP(hipMemcpy(h.data(), c->d_counts, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
  for (int i = 0; i < c->n_pairs; ++i) {
    if (h[2 * i + 1]) {
      set_error("a census count does not fit in 64 bits");
      return GZ_EOVERFLOW;
    }
    if (counts) counts[i] = h[2 * i];
  }
  if (ms) *ms = t;
  return GZ_OK;
}

// Autotuning: task granularity of 3-vertex patterns and of larger ones, and
// tasks per queue pop; each candidate is rebuilt, captured and replayed
// twice, the fastest kept.
gz_status census_tune(void* p, int32_t* params, float* best_ms) {
  auto* c = (gz_census_impl*)p;
  const int c3s[] = {8, 32, 128};
  const int c45s[] = {1, 4, 16};
  const int batches[] = {1, 4};
  float best = -1.0f;
  int b3 = c->chunk3, b45 = c->chunk45, bb = c->batch;
  for (int x3 : c3s)
    for (int x45 : c45s)
      for (int xb : batches) {
        c->chunk3 = x3;
        c->chunk45 = x45;
        c->batch = xb;
        gz_status rc = census_build(c);
        if (rc) return rc;
        float t1 = 0.0f, t2 = 0.0f;
        rc = census_launch(c, &t1);
        if (!rc) rc = census_launch(c, &t2);
        if (rc) return rc;
        const float t = std::min(t1, t2);
        if (best < 0.0f || t < best) {
          best = t;
          b3 = x3;
          b45 = x45;
          bb = xb;
        }
      }
  c->chunk3 = b3;
  c->chunk45 = b45;
  c->batch = bb;
  gz_status rc = census_build(c);
  if (rc) return rc;
  if (params) {
    params[0] = b3;
    params[1] = b45;
    params[2] = bb;
  }
  if (best_ms) *best_ms = best;
  return GZ_OK;
}

void free_graph_tasks(gz_graph* g) {
  for (auto& kv : g->task_cache) (void)hipFree(kv.second.prefix);
  g->task_cache.clear();
  free_clique_lists(&g->clique_all);
  g->clique_ready = false;
  for (HubMaps& hm : g->hub_cache)
    if (hm.bits) (void)hipFree(hm.bits);
  g->hub_cache.clear();
}

}  // namespace gz
