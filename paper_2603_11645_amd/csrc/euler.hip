// euler.hip -- Euler-tour rooting of a spanning forest (Sec. III-D).
//
// Arc numbering: the forest edge held by slot x gives twin arcs 2x = (tu->tv)
// and 2x+1 = (tv->tu), so rev(e) = e ^ 1 and no compaction pass is needed (a
// slot whose vertex stayed a component root is empty).  The paper sorts the
// arcs only to make every vertex's out-arcs form one list; any cyclic order of
// them yields a valid tour, so the per-vertex lists are built here by linking
// each arc in front of its source's list with one atomic exchange
// (head[v], next[e]).
//
// Successor (the equation of Sec. III-D): succ(e) = next(rev e) if that is not
// -1, else the first arc of from(rev e) = to(e).  Cycle breaking: the arc whose
// successor would wrap around to the root's first out-arc is the reverse of
// the root's last out-arc, i.e. an arc e into a root with next(rev e) = -1;
// it gets succ -1.  Both rules are applied in one pass that also initialises
// the ranking words.
//
// List ranking (Wyllie pointer jumping): each arc holds a packed 64-bit word
// (succ in the low half, hops-to-succ in the high half); a round replaces it by
// (succ of succ, own hops + hops of succ).  The word is read and written with
// single 64-bit accesses, so every read sees a consistent pair and rounds can
// update in place: a read of an already-advanced neighbour only moves the
// reader further.  After ceil(log2 L) rounds every word holds (-1, distance to
// the tail of its list).
//
// Parent rule: of the twins e=(u->v) and rev e, the one with the larger
// distance to the tail comes first in the tour; it is the downward traversal,
// so P[v] = u.  Component roots get P[r] = r.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

__device__ __forceinline__ uint64_t pack_rank(int32_t succ, uint32_t hops) {
  return ((uint64_t)hops << 32) | (uint32_t)succ;
}

__device__ __forceinline__ bool is_root(int32_t v, const int32_t *cc, const int32_t *comp_root) {
  const int32_t c = cc[v];
  const int32_t d = comp_root[c];
  return d == v || (d == -1 && c == v);
}

// Designated roots: claim their component, P[r] = r.
__global__ void k_mark_roots(const int32_t *__restrict__ roots, int32_t nroots, int64_t n,
                             const int32_t *__restrict__ cc, int32_t *comp_root, int32_t *parent,
                             int32_t *counters) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nroots) return;
  const int32_t r = roots[i];
  if (r < 0 || r >= n) {
    atomicOr(&counters[kCntRangeErr], 1);
    return;
  }
  const int32_t old = atomicCAS(&comp_root[cc[r]], -1, r);
  if (old != -1 && old != r) atomicOr(&counters[kCntRootErr], 1);
  parent[r] = r;
}

// Per-vertex out-arc lists: next[e] = previous head of src(e), head = e.
__global__ __launch_bounds__(kBlock) void k_link(int64_t slots, const int32_t *__restrict__ tu,
                                                 const int32_t *__restrict__ tv, int32_t *head,
                                                 int32_t *next) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= slots) return;
  const int32_t a = tu[x];
  int2 nx = make_int2(-1, -1);
  if (a >= 0) {
    const int32_t b = tv[x];
    nx.x = atomicExch(&head[a], (int32_t)(2 * x));
    nx.y = atomicExch(&head[b], (int32_t)(2 * x + 1));
  }
  reinterpret_cast<int2 *>(next)[x] = nx;
}

// Successor + cycle break + rank init for both arcs of a slot.
__global__ __launch_bounds__(kBlock) void k_succ(int64_t slots, const int32_t *__restrict__ tu,
                                                 const int32_t *__restrict__ tv,
                                                 const int32_t *__restrict__ head,
                                                 const int32_t *__restrict__ next,
                                                 const int32_t *__restrict__ cc,
                                                 const int32_t *__restrict__ comp_root,
                                                 uint64_t *rank) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= slots) return;
  const int32_t a = tu[x];
  ulonglong2 out;
  if (a < 0) {
    out.x = pack_rank(-1, 0);
    out.y = pack_rank(-1, 0);
  } else {
    const int32_t b = tv[x];
    const int2 nx = reinterpret_cast<const int2 *>(next)[x];
    // arc 2x = a->b, its reverse is 2x+1 = b->a
    int32_t s0 = nx.y;
    if (s0 == -1) s0 = is_root(b, cc, comp_root) ? -1 : head[b];
    int32_t s1 = nx.x;
    if (s1 == -1) s1 = is_root(a, cc, comp_root) ? -1 : head[a];
    out.x = pack_rank(s0, s0 >= 0 ? 1u : 0u);
    out.y = pack_rank(s1, s1 >= 0 ? 1u : 0u);
  }
  reinterpret_cast<ulonglong2 *>(rank)[x] = out;
}

__global__ __launch_bounds__(kBlock) void k_rank_init(int64_t A, const int32_t *__restrict__ succ,
                                                      uint64_t *rank) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A) return;
  int32_t s = succ[e];
  if (s < 0 || s >= A) s = -1;   // out-of-range successors end the list (no wild gathers)
  rank[e] = pack_rank(s, s >= 0 ? 1u : 0u);
}

// One pointer-jumping round over A words, EPT words per thread; all gathers of
// a thread are issued before any of them is consumed.
template <int EPT>
__global__ __launch_bounds__(kBlock) void k_rank_round(int64_t A, uint64_t *rank) {
  const int64_t base = (int64_t)blockIdx.x * (kBlock * EPT) + threadIdx.x;
  uint64_t me[EPT], nb[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int64_t i = base + (int64_t)j * kBlock;
    me[j] = i < A ? rank[i] : pack_rank(-1, 0);
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int32_t s = (int32_t)(uint32_t)me[j];
    nb[j] = s >= 0 ? rank[s] : 0ull;
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int32_t s = (int32_t)(uint32_t)me[j];
    if (s >= 0) {
      const uint64_t hops = (me[j] >> 32) + (nb[j] >> 32);
      rank[base + (int64_t)j * kBlock] = (hops << 32) | (nb[j] & 0xffffffffull);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_rank_extract(int64_t A, const uint64_t *__restrict__ rank,
                                                         int32_t *dist) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < A) dist[e] = (int32_t)(rank[e] >> 32);
}

// Parents from tour order (slots) + default component roots (vertices).
__global__ __launch_bounds__(kBlock) void k_parent(int64_t slots, int64_t n,
                                                   const int32_t *__restrict__ tu,
                                                   const int32_t *__restrict__ tv,
                                                   const uint64_t *__restrict__ rank,
                                                   const int32_t *__restrict__ cc,
                                                   const int32_t *__restrict__ comp_root,
                                                   int32_t *parent, int32_t *counters) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < slots) {
    const int32_t a = tu[x];
    if (a >= 0) {
      const int32_t b = tv[x];
      const ulonglong2 r = reinterpret_cast<const ulonglong2 *>(rank)[x];
      const uint32_t d0 = (uint32_t)(r.x >> 32), d1 = (uint32_t)(r.y >> 32);
      if (d0 > d1) parent[b] = a;   // a->b comes first: it descends
      else parent[a] = b;           // b->a comes first: b is a's parent
    }
  }
  bool comp = false;
  if (x < n) {
    comp = cc[x] == (int32_t)x;
    if (comp && comp_root[x] == -1) parent[x] = (int32_t)x;
  }
  wave_count(comp, &counters[kCntComponents]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int rank_rounds_for(int64_t max_list_len) {
  int r = 0;
  while (((int64_t)1 << r) < max_list_len) ++r;
  return r;
}

rst_status enqueue_mark_roots(rst_ctx *ctx, const int32_t *roots, int32_t nroots, int64_t n,
                              const int32_t *cc, int32_t *comp_root, int32_t *parent,
                              int32_t *counters) {
  if (nroots <= 0) return RST_OK;
  hipLaunchKernelGGL(k_mark_roots, dim3(grid_for(nroots, kBlock)), dim3(kBlock), 0, ctx->stream,
                     roots, nroots, n, cc, comp_root, parent, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_link(rst_ctx *ctx, int64_t slots, const int32_t *tu, const int32_t *tv,
                        int32_t *head, int32_t *next) {
  if (slots <= 0) return RST_OK;
  hipLaunchKernelGGL(k_link, dim3(grid_for(slots, kBlock)), dim3(kBlock), 0, ctx->stream, slots,
                     tu, tv, head, next);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_succ(rst_ctx *ctx, int64_t slots, const int32_t *tu, const int32_t *tv,
                        const int32_t *head, const int32_t *next, const int32_t *cc,
                        const int32_t *comp_root, uint64_t *rank) {
  if (slots <= 0) return RST_OK;
  hipLaunchKernelGGL(k_succ, dim3(grid_for(slots, kBlock)), dim3(kBlock), 0, ctx->stream, slots,
                     tu, tv, head, next, cc, comp_root, rank);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_rank_init(rst_ctx *ctx, int64_t A, const int32_t *succ, uint64_t *rank) {
  if (A <= 0) return RST_OK;
  hipLaunchKernelGGL(k_rank_init, dim3(grid_for(A, kBlock)), dim3(kBlock), 0, ctx->stream, A,
                     succ, rank);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

template <int EPT>
static rst_status launch_rounds(rst_ctx *ctx, int64_t A, uint64_t *rank, int rounds) {
  const unsigned grid = grid_for(A, kBlock * EPT);
  for (int r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(k_rank_round<EPT>, dim3(grid), dim3(kBlock), 0, ctx->stream, A, rank);
    RST_HIP(hipGetLastError());
  }
  return RST_OK;
}

rst_status enqueue_rank_rounds(rst_ctx *ctx, int64_t A, uint64_t *rank, int rounds,
                               hipEvent_t ev_begin, hipEvent_t ev_end) {
  if (ev_begin) RST_HIP(hipEventRecord(ev_begin, ctx->stream));
  if (A > 0 && rounds > 0) {
    switch (ctx->opt.rank_elems_per_thread) {
      case 1: RST_TRY(launch_rounds<1>(ctx, A, rank, rounds)); break;
      case 2: RST_TRY(launch_rounds<2>(ctx, A, rank, rounds)); break;
      case 8: RST_TRY(launch_rounds<8>(ctx, A, rank, rounds)); break;
      default: RST_TRY(launch_rounds<4>(ctx, A, rank, rounds)); break;
    }
  }
  if (ev_end) RST_HIP(hipEventRecord(ev_end, ctx->stream));
  return RST_OK;
}

rst_status enqueue_rank_extract(rst_ctx *ctx, int64_t A, const uint64_t *rank, int32_t *dist) {
  if (A <= 0) return RST_OK;
  hipLaunchKernelGGL(k_rank_extract, dim3(grid_for(A, kBlock)), dim3(kBlock), 0, ctx->stream, A,
                     rank, dist);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                          const int32_t *tv, const uint64_t *rank, const int32_t *cc,
                          const int32_t *comp_root, int32_t *parent, int32_t *counters) {
  const int64_t items = slots > n ? slots : n;
  hipLaunchKernelGGL(k_parent, dim3(grid_for(items, kBlock)), dim3(kBlock), 0, ctx->stream, slots,
                     n, tu, tv, rank, cc, comp_root, parent, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

}  // namespace rst
