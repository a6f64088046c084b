// Graph preparation on the device: the same normalisation and degree
// reindex (Section 6, first technique) as the host path, by sorting.
//
// 1. Every input edge {u, v}, u != v, becomes the two packed keys
//    (u << B) | v and (v << B) | u, B = bit length of n; self-loops and
//    (flagged) out-of-range endpoints become a sentinel that sorts last.
// 2. A radix sort over 2B bits and a unique pass give the symmetric,
//    duplicate-free, row-sorted edge list; rows start where a binary search
//    for (u << B) lands.
// 3. Reindex: vertex keys ((2^32 - 1 - degree) << 32) | id sorted ascending
//    give the order by decreasing degree, ties by increasing id; edges are
//    relabelled and sorted once more.
// 4. lo[v], the number of neighbours with a smaller id, is a binary search
//    for v in its own row.
// The result stays resident for counting and is copied back to the host
// handle, which the schedule-independent host code (task prefixes, root
// lists, export) reads.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_select.hpp>

#include <string>
#include <vector>

#include "gz_internal.h"

namespace gz {
namespace prep {

constexpr int TPB = 256;

__device__ __forceinline__ uint64_t pack(uint32_t u, uint32_t v, int B) {
  return ((uint64_t)u << B) | (uint64_t)v;
}

__global__ void k_edge_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                            int64_t m, int32_t n, int B, uint64_t sentinel,
                            uint64_t* __restrict__ keys, unsigned int* __restrict__ bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = src[i], v = dst[i];
    uint64_t k0 = sentinel, k1 = sentinel;
    if (u < 0 || u >= n || v < 0 || v >= n) {
      atomicOr(bad, 1u);
    } else if (u != v) {
      k0 = pack((uint32_t)u, (uint32_t)v, B);
      k1 = pack((uint32_t)v, (uint32_t)u, B);
    }
    keys[2 * i] = k0;
    keys[2 * i + 1] = k1;
  }
}

// rowptr[u] = first key index with row >= u, for u in [0, n]
__global__ void k_row_starts(const uint64_t* __restrict__ keys, int64_t cnt, int32_t n, int B,
                             int32_t* __restrict__ rowptr) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t target = (uint64_t)u << B;
    int64_t lo = 0, hi = cnt;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < target) lo = mid + 1; else hi = mid;
    }
    rowptr[u] = (int32_t)lo;
  }
}

__global__ void k_cols(const uint64_t* __restrict__ keys, int64_t cnt, int B,
                       int32_t* __restrict__ col) {
  const uint64_t mask = ((uint64_t)1 << B) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x)
    col[i] = (int32_t)(keys[i] & mask);
}

__global__ void k_vertex_keys(const int32_t* __restrict__ rowptr, int32_t n,
                              uint64_t* __restrict__ vkeys) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t deg = (uint32_t)(rowptr[v + 1] - rowptr[v]);
    vkeys[v] = ((uint64_t)(0xFFFFFFFFu - deg) << 32) | (uint64_t)v;
  }
}

__global__ void k_ranks(const uint64_t* __restrict__ sorted_vkeys, int32_t n,
                        int32_t* __restrict__ new_of_old, int32_t* __restrict__ old_of_new) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)(sorted_vkeys[r] & 0xFFFFFFFFull);
    new_of_old[v] = (int32_t)r;
    old_of_new[r] = v;
  }
}

__global__ void k_relabel(const uint64_t* __restrict__ keys, int64_t cnt, int B,
                          const int32_t* __restrict__ new_of_old, uint64_t* __restrict__ out) {
  const uint64_t mask = ((uint64_t)1 << B) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = (uint32_t)(keys[i] >> B), v = (uint32_t)(keys[i] & mask);
    out[i] = pack((uint32_t)new_of_old[u], (uint32_t)new_of_old[v], B);
  }
}

__global__ void k_identity(int32_t n, int32_t* __restrict__ p) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    p[v] = (int32_t)v;
}

__global__ void k_lo(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                     int32_t n, int32_t* __restrict__ lo) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    int32_t a = rowptr[v], b = rowptr[v + 1];
    const int32_t start = a;
    while (a < b) {
      const int32_t mid = (a + b) >> 1;
      if (col[mid] < (int32_t)v) a = mid + 1; else b = mid;
    }
    lo[v] = a - start;
  }
}

unsigned grid_for(int64_t work) {
  const int64_t b = (work + TPB - 1) / TPB;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16));
}

// Device buffers of one preparation, freed on every exit.
struct Scratch {
  std::vector<void*> p;
  ~Scratch() {
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
  template <typename T>
  bool alloc(T** out, size_t count) {
    *out = nullptr;
    if (hipMalloc((void**)out, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) return false;
    p.push_back(*out);
    return true;
  }
  void release(void* q) {
    for (void*& x : p)
      if (x == q) x = nullptr;
  }
};

}  // namespace prep

#define GZ_PREP_HIP(call)                                                 \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      set_error(std::string("device preparation: ") + #call + ": " +      \
                hipGetErrorString(e_));                                   \
      return GZ_EDEVICE;                                                  \
    }                                                                     \
  } while (0)

// Prepare a raw edge list on the current device.  src/dst are device
// pointers when `device_inputs`, else host pointers (uploaded here).  On
// success g->d_rowptr / d_col / d_lo hold the prepared graph and g->host a
// copy of it (with old_of_new); statistics are left to the caller.
gz_status device_prepare_edges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                               bool device_inputs, bool reindex, hipStream_t st, gz_graph* g) {
  using namespace prep;
  if (n < 0 || m < 0) {
    set_error("n or m out of range");
    return GZ_EINVAL;
  }
  if (m >= (int64_t)1 << 31) {  // 2m keys must fit the 32-bit offsets of the unique pass
    set_error("device preparation takes fewer than 2^31 input edges");
    return GZ_EINVAL;
  }
  Scratch s;
  const int B = n > 0 ? 32 - __builtin_clz((unsigned)n) : 1;  // bit length of n
  const uint64_t sentinel = ((uint64_t)1 << (2 * B)) - 1;
  const int64_t nk = 2 * m;
  const int32_t *ds = src, *dd = dst;
  if (!device_inputs && m > 0) {
    int32_t *us = nullptr, *ud = nullptr;
    if (!s.alloc(&us, (size_t)m) || !s.alloc(&ud, (size_t)m)) {
      set_error("device allocation failed");
      return GZ_ENOMEM;
    }
    GZ_PREP_HIP(hipMemcpyAsync(us, src, sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
    GZ_PREP_HIP(hipMemcpyAsync(ud, dst, sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
    ds = us;
    dd = ud;
  }
  uint64_t *k0 = nullptr, *k1 = nullptr;
  unsigned int* d_bad = nullptr;
  unsigned int* d_cnt = nullptr;
  int32_t *rowptr = nullptr, *col = nullptr, *lo = nullptr;
  if (!s.alloc(&k0, (size_t)nk) || !s.alloc(&k1, (size_t)nk) || !s.alloc(&d_bad, 1) ||
      !s.alloc(&d_cnt, 1) || !s.alloc(&rowptr, (size_t)n + 1) || !s.alloc(&lo, (size_t)n)) {
    set_error("device allocation failed");
    return GZ_ENOMEM;
  }
  GZ_PREP_HIP(hipMemsetAsync(d_bad, 0, sizeof(unsigned int), st));
  int64_t cnt = 0;
  if (m > 0) {
    hipLaunchKernelGGL(k_edge_keys, dim3(grid_for(m)), dim3(TPB), 0, st, ds, dd, m, n, B,
                       sentinel, k0, d_bad);
    GZ_PREP_HIP(hipGetLastError());
    unsigned int bad = 0;
    GZ_PREP_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, st));
    GZ_PREP_HIP(hipStreamSynchronize(st));
    if (bad) {
      set_error("edge endpoint out of range [0, n)");
      return GZ_EINVAL;
    }
    // sort, then drop duplicates and the trailing sentinel run
    size_t tmp_bytes = 0, tmp2 = 0;
    GZ_PREP_HIP(rocprim::radix_sort_keys(nullptr, tmp_bytes, k0, k1, (size_t)nk, 0, 2 * B, st));
    GZ_PREP_HIP(rocprim::unique(nullptr, tmp2, k1, k0, d_cnt, (size_t)nk,
                                rocprim::equal_to<uint64_t>(), st));
    void* tmp = nullptr;
    if (!s.alloc((char**)&tmp, std::max(tmp_bytes, tmp2))) {
      set_error("device allocation failed");
      return GZ_ENOMEM;
    }
    size_t b1 = std::max(tmp_bytes, tmp2);
    GZ_PREP_HIP(rocprim::radix_sort_keys(tmp, b1, k0, k1, (size_t)nk, 0, 2 * B, st));
    b1 = std::max(tmp_bytes, tmp2);
    GZ_PREP_HIP(rocprim::unique(tmp, b1, k1, k0, d_cnt, (size_t)nk,
                                rocprim::equal_to<uint64_t>(), st));
    unsigned int ucnt = 0;
    uint64_t last = 0;
    GZ_PREP_HIP(hipMemcpyAsync(&ucnt, d_cnt, sizeof(ucnt), hipMemcpyDeviceToHost, st));
    GZ_PREP_HIP(hipStreamSynchronize(st));
    if (ucnt > 0) {
      GZ_PREP_HIP(hipMemcpyAsync(&last, k0 + (ucnt - 1), sizeof(last), hipMemcpyDeviceToHost, st));
      GZ_PREP_HIP(hipStreamSynchronize(st));
    }
    cnt = (int64_t)ucnt - ((ucnt > 0 && last == sentinel) ? 1 : 0);
    if (cnt > INT32_MAX) {
      set_error("graph has 2^31 or more neighbour entries");
      return GZ_EINVAL;
    }
  }
  // k0[0, cnt): sorted unique keys of the graph in the caller's ids
  if (!s.alloc(&col, (size_t)cnt)) {
    set_error("device allocation failed");
    return GZ_ENOMEM;
  }
  hipLaunchKernelGGL(k_row_starts, dim3(grid_for((int64_t)n + 1)), dim3(TPB), 0, st, k0, cnt, n,
                     B, rowptr);
  GZ_PREP_HIP(hipGetLastError());
  int32_t *new_of_old = nullptr, *old_of_new = nullptr;
  if (!s.alloc(&new_of_old, (size_t)n) || !s.alloc(&old_of_new, (size_t)n)) {
    set_error("device allocation failed");
    return GZ_ENOMEM;
  }
  if (reindex && n > 0) {
    uint64_t *vk0 = nullptr, *vk1 = nullptr;
    if (!s.alloc(&vk0, (size_t)n) || !s.alloc(&vk1, (size_t)n)) {
      set_error("device allocation failed");
      return GZ_ENOMEM;
    }
    hipLaunchKernelGGL(k_vertex_keys, dim3(grid_for(n)), dim3(TPB), 0, st, rowptr, n, vk0);
    GZ_PREP_HIP(hipGetLastError());
    size_t tb = 0;
    GZ_PREP_HIP(rocprim::radix_sort_keys(nullptr, tb, vk0, vk1, (size_t)n, 0, 64, st));
    void* tmp = nullptr;
    if (!s.alloc((char**)&tmp, tb)) {
      set_error("device allocation failed");
      return GZ_ENOMEM;
    }
    GZ_PREP_HIP(rocprim::radix_sort_keys(tmp, tb, vk0, vk1, (size_t)n, 0, 64, st));
    hipLaunchKernelGGL(k_ranks, dim3(grid_for(n)), dim3(TPB), 0, st, vk1, n, new_of_old,
                       old_of_new);
    GZ_PREP_HIP(hipGetLastError());
    if (cnt > 0) {
      hipLaunchKernelGGL(k_relabel, dim3(grid_for(cnt)), dim3(TPB), 0, st, k0, cnt, B,
                         new_of_old, k1);
      GZ_PREP_HIP(hipGetLastError());
      size_t tb2 = 0;
      GZ_PREP_HIP(rocprim::radix_sort_keys(nullptr, tb2, k1, k0, (size_t)cnt, 0, 2 * B, st));
      void* tmp2 = nullptr;
      if (!s.alloc((char**)&tmp2, tb2)) {
        set_error("device allocation failed");
        return GZ_ENOMEM;
      }
      GZ_PREP_HIP(rocprim::radix_sort_keys(tmp2, tb2, k1, k0, (size_t)cnt, 0, 2 * B, st));
    }
    hipLaunchKernelGGL(k_row_starts, dim3(grid_for((int64_t)n + 1)), dim3(TPB), 0, st, k0, cnt,
                       n, B, rowptr);
    GZ_PREP_HIP(hipGetLastError());
  } else if (n > 0) {
    hipLaunchKernelGGL(k_identity, dim3(grid_for(n)), dim3(TPB), 0, st, n, old_of_new);
    GZ_PREP_HIP(hipGetLastError());
  }
  if (cnt > 0) {
    hipLaunchKernelGGL(k_cols, dim3(grid_for(cnt)), dim3(TPB), 0, st, k0, cnt, B, col);
    GZ_PREP_HIP(hipGetLastError());
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_lo, dim3(grid_for(n)), dim3(TPB), 0, st, rowptr, col, n, lo);
    GZ_PREP_HIP(hipGetLastError());
  }
  // host copy of the prepared graph
  HostGraph& h = g->host;
  h.n = n;
  h.rowptr.resize((size_t)n + 1);
  h.col.resize((size_t)cnt);
  h.lo.resize((size_t)n);
  h.old_of_new.resize((size_t)n);
  GZ_PREP_HIP(hipMemcpyAsync(h.rowptr.data(), rowptr, sizeof(int32_t) * ((size_t)n + 1),
                             hipMemcpyDeviceToHost, st));
  if (cnt)
    GZ_PREP_HIP(hipMemcpyAsync(h.col.data(), col, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost,
                               st));
  if (n) {
    GZ_PREP_HIP(hipMemcpyAsync(h.lo.data(), lo, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    GZ_PREP_HIP(hipMemcpyAsync(h.old_of_new.data(), old_of_new, sizeof(int32_t) * n,
                               hipMemcpyDeviceToHost, st));
  }
  GZ_PREP_HIP(hipStreamSynchronize(st));
  GZ_PREP_HIP(hipGetDevice(&g->device));
  // the prepared arrays now belong to the handle
  g->d_rowptr = rowptr;
  g->d_col = col;
  g->d_lo = lo;
  s.release(rowptr);
  s.release(col);
  s.release(lo);
  return GZ_OK;
}

}  // namespace gz
