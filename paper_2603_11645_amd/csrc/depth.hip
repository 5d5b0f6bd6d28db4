// depth.hip -- depth of every vertex of a rooted forest by its Euler tour
// (the tree-depth comparison of Sec. IV-B, Fig. 2; the tour of Sec. III-D).
//
// The forest is given by its parent array.  Non-root v holds the edge
// (P[v], v) in slot v, as arcs 2v and 2v+1: the one whose id has an even
// number of one bits goes down (P[v] -> v), the other up (v -> P[v]), see
// tour_down; every vertex's out-arcs form a list (atomic exchange), the tour
// successor is next(rev e) or, at the end of a list, the first out-arc of the
// arc's head, and the tour of each tree starts at its root's first out-arc and
// ends at the arc whose successor would wrap around to it.  Along a tour the
// arcs weigh +1 (down) and -1 (up); the depth of v is the sum of the weights
// up to and including its down arc, and since a tour sums to zero, that is
// minus the sum of the weights after it.  Each arc's word holds (successor,
// weight of the successor), so the weighted distance to the tail computed
// by the sparse ruling set of glrank.hip is exactly that sum.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

// Maximum of d over the workgroup into *out: one atomic per workgroup at
// most, and none when the value read beforehand is already as large (the
// maximum only grows, so a stale read costs just an atomic).  One atomic per
// workgroup on the single word still serialised the pass: 1.5 ms for 65536
// workgroups.  Called by all threads.
template <int B>
__device__ __forceinline__ void block_max_to(int32_t d, int32_t *out) {
  __shared__ int32_t s_max[B / 64];
  for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o, 64));
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t m = s_max[0];
    for (int w = 1; w < B / 64; ++w) m = max(m, s_max[w]);
    if (m > __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(out, m);
  }
}

__device__ __forceinline__ bool depth_is_root(int32_t v, int32_t p, int64_t n) {
  return p == v || p < 0 || p >= n;   // out-of-range parents are taken as roots
}

// The down arc of slot x: 2x when x has an even number of one bits, else
// 2x+1 (the up arc is the other one), so an arc goes down iff its id has an
// even number of one bits.  The ruling set's rulers are the arc ids divisible
// by its stride; with every down arc even they were all down arcs, a climb of
// up arcs held none, and one lane walked all of it (a chain-like tree's tour:
// 2.8 ms against 1.1 ms for a tour of the same length numbered by hooking).
__device__ __forceinline__ int32_t tour_down(int64_t x) {
  return (int32_t)(2 * x + (__popcll((unsigned long long)x) & 1));
}
__device__ __forceinline__ bool tour_arc_down(int32_t e) {
  return (__popc((uint32_t)e) & 1) == 0;
}

// Out-arc lists of the forest of parent edges, in two passes: every non-root
// x's list starts as its up arc alone (which so stays last), then every
// child puts its down arc in front of its parent's list.  (An exchange for
// the up arc as well cost a chain-like tree's linking a third of its time.)
template <int B>
__global__ __launch_bounds__(B) void k_depth_heads(int64_t n, const int32_t *__restrict__ parent,
                                                   int32_t *head) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  head[x] = depth_is_root((int32_t)x, parent[x], n) ? -1 : tour_down(x) ^ 1;
}

template <int B>
__global__ __launch_bounds__(B) void k_depth_link(int64_t n, const int32_t *__restrict__ parent,
                                                  int32_t *head, int32_t *next) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const int32_t p = parent[x];
  int2 nx = make_int2(-1, -1);
  if (!depth_is_root((int32_t)x, p, n)) {
    const int32_t dn = tour_down(x);
    const int32_t nd = atomicExch(&head[p], dn);   // p -> x; x -> p ends x's list
    nx = (dn & 1) ? make_int2(-1, nd) : make_int2(nd, -1);   // next[2x], next[2x+1]
  }
  reinterpret_cast<int2 *>(next)[x] = nx;
}

// weight of the successor arc, 0 past the tail: depth (kPre false) +1 down,
// -1 up; preorder (kPre true) 1 down, 0 up
template <bool kPre>
__device__ __forceinline__ uint64_t depth_word(int32_t succ) {
  const uint32_t w = succ < 0 ? 0u : (tour_arc_down(succ) ? 1u : (kPre ? 0u : 0xffffffffu));
  return ((uint64_t)w << 32) | (uint32_t)succ;
}

// Successors of the down and the up arc of non-root x (child of p): after
// p -> x comes the arc after x -> p in x's list, or x's first (x's list holds
// x -> p); after x -> p the arc after p -> x in p's list, or p's first unless
// p roots its tree (the end of the tour).
__device__ __forceinline__ int2 tour_succ(int64_t x, int32_t p, int64_t n,
                                          const int32_t *__restrict__ parent,
                                          const int32_t *__restrict__ head,
                                          const int32_t *__restrict__ next) {
  const int2 nx = reinterpret_cast<const int2 *>(next)[x];
  const bool odd = tour_down(x) & 1;
  const int32_t after_down = odd ? nx.y : nx.x, after_up = odd ? nx.x : nx.y;
  int2 s;
  s.x = after_up != -1 ? after_up : head[x];
  s.y = after_down;
  if (s.y == -1) s.y = depth_is_root(p, parent[p], n) ? -1 : head[p];
  return s;
}

// Level-1 words (successor, weight) of both arcs of every slot, and the list
// heads (the first out-arc of every root with arcs).
template <bool kPre>
__device__ __forceinline__ void tour_words(int64_t n, const int32_t *__restrict__ parent,
                                           const int32_t *__restrict__ head,
                                           const int32_t *__restrict__ next, uint64_t *w,
                                           int32_t *heads, int64_t hcap, int32_t *counters) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool is_head = false;
  int32_t h = -1;
  if (x < n) {
    const int32_t p = parent[x];
    ulonglong2 out = make_ulonglong2(0x00000000fffffffeull, 0x00000000fffffffeull);   // no list
    if (depth_is_root((int32_t)x, p, n)) {
      h = head[x];
      is_head = h >= 0;
    } else {
      const int2 sc = tour_succ(x, p, n, parent, head, next);
      const uint64_t wd = depth_word<kPre>(sc.x), wu = depth_word<kPre>(sc.y);
      if (tour_down(x) & 1) { out.x = wu; out.y = wd; } else { out.x = wd; out.y = wu; }
    }
    reinterpret_cast<ulonglong2 *>(w)[x] = out;
  }
  const int slot = wave_append(is_head, &counters[kCntGHeads]);
  if (is_head && slot < hcap) heads[slot] = h;
}

template <int B>
__global__ __launch_bounds__(B) void k_depth_words(int64_t n, const int32_t *__restrict__ parent,
                                                   const int32_t *__restrict__ head,
                                                   const int32_t *__restrict__ next, uint64_t *w,
                                                   int32_t *heads, int64_t hcap, int32_t *counters) {
  tour_words<false>(n, parent, head, next, w, heads, hcap, counters);
}

// Preorder ranking in 32-bit words: each arc's word is its successor (-2 for
// an arc of no list), the weight (1 down, 0 up) following from the
// successor's id in the walk (tour_arc_down); list heads as above.
template <int B>
__global__ __launch_bounds__(B) void k_pre_words32(int64_t n, const int32_t *__restrict__ parent,
                                                   const int32_t *__restrict__ head,
                                                   const int32_t *__restrict__ next, int32_t *w,
                                                   int32_t *heads, int64_t hcap, int32_t *counters) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool is_head = false;
  int32_t h = -1;
  if (x < n) {
    const int32_t p = parent[x];
    int2 out = make_int2(-2, -2);
    if (depth_is_root((int32_t)x, p, n)) {
      h = head[x];
      is_head = h >= 0;
    } else {
      const int2 sc = tour_succ(x, p, n, parent, head, next);
      out = (tour_down(x) & 1) ? make_int2(sc.y, sc.x) : sc;
    }
    reinterpret_cast<int2 *>(w)[x] = out;
  }
  const int slot = wave_append(is_head, &counters[kCntGHeads]);
  if (is_head && slot < hcap) heads[slot] = h;
}

template <int B>
__global__ __launch_bounds__(B) void k_pre_words(int64_t n, const int32_t *__restrict__ parent,
                                                 const int32_t *__restrict__ head,
                                                 const int32_t *__restrict__ next, uint64_t *w,
                                                 int32_t *heads, int64_t hcap, int32_t *counters) {
  tour_words<true>(n, parent, head, next, w, heads, hcap, counters);
}

// depth[x] = -(weighted distance after x's down arc), 0 at roots; the
// largest depth goes to counters[kCntDepthMax].
template <int B>
__global__ __launch_bounds__(B) void k_depth_out(int64_t n, const int32_t *__restrict__ parent,
                                                 const uint64_t *__restrict__ w,
                                                 const uint32_t *__restrict__ d1, int64_t rw1_cap,
                                                 int32_t *depth, int32_t *counters) {
  if (counters[kCntGOverflow]) return;   // block-uniform: the caller falls back
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t d = 0;
  if (x < n) {
    if (!depth_is_root((int32_t)x, parent[x], n)) {
      const uint64_t c = w[tour_down(x)];
      const uint32_t rid = (uint32_t)c;
      const uint32_t dist = rid < rw1_cap ? d1[rid] - (uint32_t)(c >> 32) : 0u;
      d = -(int32_t)dist;
    }
    depth[x] = d;
  }
  block_max_to<B>(d, &counters[kCntDepthMax]);
}

// Fallback after counters[kCntGOverflow] (more trees than the ruling set
// holds): Wyllie rounds over the same weighted words, then the same output.
template <int B>
__global__ __launch_bounds__(B) void k_depth_out_rounds(int64_t n, const int32_t *__restrict__ parent,
                                                        const uint64_t *__restrict__ w,
                                                        int32_t *depth, int32_t *counters) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t d = 0;
  if (x < n) {
    if (!depth_is_root((int32_t)x, parent[x], n)) d = -(int32_t)(uint32_t)(w[tour_down(x)] >> 32);
    depth[x] = d;
  }
  block_max_to<B>(d, &counters[kCntDepthMax]);
}

// Preorder number and subtree size of every vertex of a tree (one root) from
// the preorder-weighted tour: D(e) = number of down arcs after arc e, so with
// x's down arc d and up arc u, pre(x) = (n - 1) - D(d) and nd(x) = D(d) -
// D(u) + 1 (the down arcs strictly inside x's excursion are its
// descendants'); the root has pre 0 and nd n.  Roots are counted into counters[kCntBccRoots].
// Each vertex's record R[x] = (parent, pre, nd, 0): one 16-byte gather
// serves a consumer that needs several of them for a random vertex.
__device__ __forceinline__ void pre_store(int64_t n, int64_t x, int32_t par, bool root, uint32_t d0,
                                          uint32_t d1, int4 *R) {
  const int32_t p = root ? 0 : (int32_t)(n - 1) - (int32_t)d0;
  const int32_t s = root ? (int32_t)n : (int32_t)d0 - (int32_t)d1 + 1;
  R[x] = make_int4(par, p, s, 0);
}

// codes (ruler << 8 | weight walked since it) of both arcs, from the 32-bit walk
template <int B>
__global__ __launch_bounds__(B) void k_pre_out(int64_t n, const int32_t *__restrict__ parent,
                                               const int32_t *__restrict__ w,
                                               const uint32_t *__restrict__ d1, int64_t rw1_cap,
                                               int4 *R, int32_t *counters) {
  if (counters[kCntGOverflow]) return;   // block-uniform: the caller falls back
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool root = false;
  if (x < n) {
    const int32_t par = parent[x];
    root = depth_is_root((int32_t)x, par, n);
    uint32_t a = 0, b = 0;
    if (!root) {
      int2 c = reinterpret_cast<const int2 *>(w)[x];
      if (tour_down(x) & 1) c = make_int2(c.y, c.x);   // (down, up)
      const uint32_t r0 = (uint32_t)c.x >> 8, r1 = (uint32_t)c.y >> 8;
      a = r0 < rw1_cap ? d1[r0] - ((uint32_t)c.x & 255u) : 0u;
      b = r1 < rw1_cap ? d1[r1] - ((uint32_t)c.y & 255u) : 0u;
    }
    pre_store(n, x, par, root, a, b, R);
  }
  wave_count(root, &counters[kCntBccRoots]);
}

template <int B>
__global__ __launch_bounds__(B) void k_pre_out_rounds(int64_t n, const int32_t *__restrict__ parent,
                                                      const uint64_t *__restrict__ w, int4 *R,
                                                      int32_t *counters) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool root = false;
  if (x < n) {
    const int32_t par = parent[x];
    root = depth_is_root((int32_t)x, par, n);
    const int32_t dn = tour_down(x);
    const uint32_t a = root ? 0u : (uint32_t)(w[dn] >> 32);
    const uint32_t b = root ? 0u : (uint32_t)(w[dn ^ 1] >> 32);
    pre_store(n, x, par, root, a, b, R);
  }
  wave_count(root, &counters[kCntBccRoots]);
}

size_t depth_ws_bytes(int64_t n, const GlistPlan &p) {
  return ws_bytes(64, 4) + ws_bytes((size_t)n, 4) + ws_bytes(2 * (size_t)n, 4) +
         ws_bytes(2 * (size_t)n, 8) + glist_ws_bytes(p);
}

rst_status run_tree_depth(rst_ctx *ctx, int64_t n, const int32_t *parent, int32_t *depth,
                          int64_t *max_depth) {
  const GlistPlan plan = glist_plan(2 * n, n / 2 + 1, ctx->opt.rank_stride);
  RST_TRY(ws_reserve(ctx, depth_ws_bytes(n, plan)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  int32_t *head = ws_take<int32_t>(ctx, n);
  int32_t *next = ws_take<int32_t>(ctx, 2 * n);
  uint64_t *w = ws_take<uint64_t>(ctx, 2 * n);
  GlistBufs gl;
  glist_take(ctx, plan, gl);
  RST_TRY(enqueue_fill(ctx, counters, 32, 0));
  RST_SWEEP(ctx, k_depth_heads, n, n, parent, head);
  RST_HIP(hipGetLastError());
  RST_SWEEP(ctx, k_depth_link, n, n, parent, head, next);
  RST_HIP(hipGetLastError());
  RST_SWEEP(ctx, k_depth_words, n, n, parent, head, next, w, gl.heads[0], plan.hcap, counters);
  RST_HIP(hipGetLastError());
  RST_TRY(enqueue_glist_rank(ctx, w, true, gl, counters));
  RST_SWEEP(ctx, k_depth_out, n, n, parent, w, gl.d1, plan.cap[1], depth, counters);
  RST_HIP(hipGetLastError());
  RST_HIP(hipMemcpyAsync(ctx->host_pinned, counters, kCntTotal * sizeof(int32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->host_pinned[kCntGOverflow]) {
    // rebuild the words (the walks overwrote them) and rank every arc
    RST_SWEEP(ctx, k_depth_words, n, n, parent, head, next, w, gl.heads[0], plan.hcap, counters);
    RST_HIP(hipGetLastError());
    RST_TRY(enqueue_rank_rounds(ctx, 2 * n, w, rank_rounds_for(2 * n), nullptr, nullptr));
    RST_SWEEP(ctx, k_depth_out_rounds, n, n, parent, w, depth, counters);
    RST_HIP(hipGetLastError());
    RST_HIP(hipMemcpyAsync(ctx->host_pinned, counters, kCntTotal * sizeof(int32_t),
                           hipMemcpyDeviceToHost, ctx->stream));
    RST_HIP(hipStreamSynchronize(ctx->stream));
  }
  if (max_depth) *max_depth = ctx->host_pinned[kCntDepthMax];
  return RST_OK;
}

rst_status run_tour_preorder(rst_ctx *ctx, int64_t n, const int32_t *parent, int4 *R,
                              int32_t *counters) {
  const GlistPlan plan = glist_plan(2 * n, n / 2 + 1, ctx->opt.rank_stride);
  int32_t *head = ws_take<int32_t>(ctx, n);
  int32_t *next = ws_take<int32_t>(ctx, 2 * n);
  uint64_t *w = ws_take<uint64_t>(ctx, 2 * n);
  GlistBufs gl;
  glist_take(ctx, plan, gl);
  RST_SWEEP(ctx, k_depth_heads, n, n, parent, head);
  RST_HIP(hipGetLastError());
  RST_SWEEP(ctx, k_depth_link, n, n, parent, head, next);
  RST_HIP(hipGetLastError());
  // 32-bit words with the weights from the arcs' ids: half the bytes of
  // (successor, weight) words under the random walk
  int32_t *w32 = reinterpret_cast<int32_t *>(w);
  RST_SWEEP(ctx, k_pre_words32, n, n, parent, head, next, w32, gl.heads[0], plan.hcap, counters);
  RST_HIP(hipGetLastError());
  RST_TRY(enqueue_glist_rank(ctx, w32, false, gl, counters, true));
  RST_SWEEP(ctx, k_pre_out, n, n, parent, w32, gl.d1, plan.cap[1], R, counters);
  RST_HIP(hipGetLastError());
  RST_HIP(hipMemcpyAsync(ctx->host_pinned, counters, kCntTotal * sizeof(int32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->host_pinned[kCntGOverflow]) {
    // rebuild the words (the walks overwrote them) and rank every arc
    RST_TRY(enqueue_fill(ctx, counters + kCntBccRoots, 1, 0));
    RST_SWEEP(ctx, k_pre_words, n, n, parent, head, next, w, gl.heads[0], plan.hcap, counters);
    RST_HIP(hipGetLastError());
    RST_TRY(enqueue_rank_rounds(ctx, 2 * n, w, rank_rounds_for(2 * n), nullptr, nullptr));
    RST_SWEEP(ctx, k_pre_out_rounds, n, n, parent, w, R, counters);
    RST_HIP(hipGetLastError());
    RST_HIP(hipMemcpyAsync(ctx->host_pinned, counters, kCntTotal * sizeof(int32_t),
                           hipMemcpyDeviceToHost, ctx->stream));
    RST_HIP(hipStreamSynchronize(ctx->stream));
  }
  return RST_OK;
}

}  // namespace rst
