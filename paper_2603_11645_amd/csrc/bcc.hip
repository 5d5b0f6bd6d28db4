// bcc.hip -- biconnected components from a rooted spanning tree: the
// downstream use of an RST that Sec. I and the opening of Sec. IV name, by
// the parallel method of Tarjan and Vishkin.
//
// Given a spanning tree T of a connected graph G rooted at r (parent P):
//  1. pre(v), nd(v): preorder number and subtree size from the Euler tour of
//     T (run_tour_preorder: the tour weighted 1 on down arcs and 0 on up
//     arcs, ranked by the sparse ruling set); v's subtree is the preorder
//     range [pre(v), pre(v) + nd(v)).
//  2. local(v) = (min, max) of pre(v) and of pre(w) over v's non-tree arcs
//     (v, w) (arcs to P(v) or to a child count as tree arcs, parallel copies
//     included; self-loops count as nothing), stored at position pre(v).
//  3. low(v), high(v): min and max of local over v's subtree range, by a
//     range-extremum structure (per 64-position block the prefix and suffix
//     extremes, a sparse table over the blocks).
//  4. An auxiliary graph on the tree edges, each named by its child vertex:
//     tree edge v and its parent's tree edge P(v) (P(v) not the root) are
//     joined when low(v) < pre(P(v)) or high(v) >= pre(P(v)) + nd(P(v)) (a
//     vertex of v's subtree has a non-tree edge leaving P(v)'s subtree);
//     non-tree edge (u, w) with pre(u) < pre(w) and w outside u's subtree
//     joins tree edges u and w.  Its connected components -- min-id hooking
//     by compare-and-swap as in the hooking pass, then pointer jumping -- are
//     the biconnected components of the tree edges, each labelled by its
//     smallest child vertex.  The joins commute, so the non-tree edges' are
//     made in step 2's pass over the arcs, which reads the same far-end
//     record, and the tree edges' after step 3.
//  5. Every arc takes its component: a tree arc (or a parallel copy) the one
//     of its child's tree edge, a non-tree arc the one of the tree edge of its
//     end with the larger preorder number; a vertex whose arcs carry two or
//     more labels is an articulation point.
#include "rst_internal.h"
#include "device_common.h"
#include "unionfind.h"

namespace rst {

constexpr int kBcChunk = 1024;   // vertices per workgroup step of the arc passes
constexpr int kBcBlock = 64;     // preorder positions per block of the extremum structure
constexpr int kBcThreads = 256;
// Vertices with more arcs than kBcHeavy leave the chunk passes: their arcs are
// cut into items of kBcSlice arcs, one workgroup step each, so that no
// workgroup walks a hub's arcs alone (on R-MAT graphs the low ids are the
// hubs, and a chunk of them held tens of millions of arcs: 43 ms on C3).
constexpr int kBcHeavy = 256;
constexpr int kBcSlice = 4096;

__device__ __forceinline__ int2 bc_comb(int2 a, int2 b) {
  return make_int2(a.x < b.x ? a.x : b.x, a.y > b.y ? a.y : b.y);
}

// Calls f(j, u, w, a) for every arc a = (u -> w) of the vertices
// [v0, v0 + kBcChunk) (j = u - v0) with at most kBcHeavy arcs: their degrees
// scanned in LDS, the union of their arcs walked with unit stride; lanes past
// the last arc call it with j = -1.  Called by all threads of the workgroup;
// ends with a barrier.
template <class OffT, class F>
__device__ __forceinline__ void bc_chunk_arcs(int64_t n, int64_t v0, const OffT *__restrict__ off,
                                              const int32_t *__restrict__ cols, int *s_scan,
                                              OffT *s_beg, int *s_wave, F f) {
  const int t = threadIdx.x;
  const int64_t v = v0 + t;
  int deg = 0;
  OffT beg = 0;
  if (v < n) {
    beg = off[v];
    const int64_t d = (int64_t)(off[v + 1] - beg);
    deg = d > kBcHeavy ? 0 : (int)d;   // heavy vertices: the item passes
  }
  s_beg[t] = beg;
  int total;
  const int excl = block_excl_scan<kBcChunk>(deg, s_wave, &total);
  s_scan[t] = excl;
  if (t == kBcChunk - 1) s_scan[kBcChunk] = excl + deg;
  __syncthreads();
  for (int b0 = 0; b0 < total; b0 += kBcChunk) {
    const int k = b0 + t;
    // every lane calls f (j = -1 past the arcs), so f may use wave operations
    int j = -1;
    int32_t w = -1;
    int64_t a = -1;
    if (k < total) {
      j = lds_upper_search(s_scan, kBcChunk, k);
      a = (int64_t)(s_beg[j] + (OffT)(k - s_scan[j]));
      w = cols[a];
    }
    f(j, (int32_t)(v0 + j), w, a);
  }
  __syncthreads();
}

// Extremes (x: min, y: max) of the lanes of each run of equal j (runs are
// contiguous: the arcs of a vertex sit on consecutive lanes), combined into
// s_x[j], s_y[j] by the run's last lane only.  Called by all lanes of the wave
// (j < 0: no vertex, value ignored).  The arcs of a hub fill whole waves:
// an LDS atomic per arc on one word serialised the pass (15 ms on a graph
// with hubs of degree 1.6e5).
__device__ __forceinline__ void bc_run_extremes(int j, int2 val, int *s_x, int *s_y) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int jo = __shfl_up(j, o, 64);
    const int2 w = make_int2(__shfl_up(val.x, o, 64), __shfl_up(val.y, o, 64));
    if (lane >= o && jo == j) val = bc_comb(val, w);
  }
  const int jn = __shfl_down(j, 1, 64);
  if (j >= 0 && (lane == kWave - 1 || jn != j)) {
    atomicMin(&s_x[j], val.x);
    atomicMax(&s_y[j], val.y);
  }
}

__device__ __forceinline__ bool bc_is_root(int32_t v, int32_t p, int64_t n) {
  return p == v || p < 0 || p >= n;
}

// The rule of step 4 for non-tree edge (u, w), seen from u: with pre(u) <
// pre(w) and w outside u's subtree it joins the tree edges of u and w.
__device__ __forceinline__ void bc_cross(int32_t u, int32_t w, const int4 &ru, const int4 &rw,
                                         int32_t *L) {
  const int64_t pu = ru.y, pw = rw.y;
  if (pu < pw && pw >= pu + ru.z) hook_join<true>(u, w, L);
}

// Step 2: local extremes, stored at each vertex's preorder position; the
// same pass over the arcs applies step 4's rule to the non-tree edges (the
// joins of step 4 commute, and both need the far end's record).  Ends with a
// device-scope release per workgroup (hooks in global memory, read on every
// XCD next).
template <class OffT>
__global__ __launch_bounds__(kBcChunk, 8) void k_bcc_local(int64_t n, const OffT *__restrict__ off,
                                                        const int32_t *__restrict__ cols,
                                                        const int4 *__restrict__ R, int2 *A,
                                                        int32_t *L, int64_t *items,
                                                        int64_t item_cap, int32_t *counters) {
  __shared__ int s_scan[kBcChunk + 1];
  __shared__ OffT s_beg[kBcChunk];
  __shared__ int s_wave[kBcChunk / kWave];
  __shared__ int s_lo[kBcChunk], s_hi[kBcChunk];
  const int t = threadIdx.x;
  const int64_t chunks = (n + kBcChunk - 1) / kBcChunk;
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int64_t v0 = c * kBcChunk, v = v0 + t;
    const int32_t pv = v < n ? R[v].y : 0;
    if (v < n) {
      // a heavy vertex's arcs become items (v, slice) for the item passes
      const int64_t d = (int64_t)(off[v + 1] - off[v]);
      if (d > kBcHeavy) {
        const int64_t ns = (d + kBcSlice - 1) / kBcSlice;
        const int64_t base = atomicAdd(&counters[kCntBccItems], (int32_t)ns);
        if (base + ns > item_cap) atomicOr(&counters[kCntRangeErr], 1);
        for (int64_t k = 0; k < ns && base + k < item_cap; ++k) items[base + k] = (v << 32) | k;
      }
    }
    s_lo[t] = pv;   // published by the scan's barriers
    s_hi[t] = pv;
    bc_chunk_arcs(n, v0, off, cols, s_scan, s_beg, s_wave,
                  [&](int j, int32_t u, int32_t w, int64_t) {
                    int2 val = make_int2(INT32_MAX, INT32_MIN);
                    // non-tree arcs only (arcs to the parent or a child, and
                    // their parallel copies, are tree arcs)
                    if (j >= 0 && w != u && w >= 0 && w < n) {
                      const int4 ru = R[u], rw = R[w];
                      if (w != ru.x && rw.x != u) {
                        val = make_int2(rw.y, rw.y);
                        bc_cross(u, w, ru, rw, L);
                      }
                    }
                    bc_run_extremes(j, val, s_lo, s_hi);
                  });
    if (v < n) {
      if (pv >= 0 && pv < n) A[pv] = make_int2(s_lo[t], s_hi[t]);
      else atomicOr(&counters[kCntRangeErr], 1);
    }
  }
  block_release_device();
}

// The arcs [a0, a1) of heavy item `it` (vertex v, slice k).
template <class OffT>
__device__ __forceinline__ int64_t bc_item(const int64_t *__restrict__ items, int64_t it,
                                           const OffT *__restrict__ off, int64_t *a0, int64_t *a1) {
  const int64_t item = items[it];
  const int64_t v = item >> 32, k = item & 0xffffffff;
  const int64_t b = (int64_t)off[v], e = (int64_t)off[v + 1];
  *a0 = b + k * kBcSlice;
  *a1 = *a0 + kBcSlice < e ? *a0 + kBcSlice : e;
  return v;
}

// extremes over the workgroup, in thread 0 (called by all threads)
__device__ __forceinline__ int2 bc_block_extremes(int2 x, int2 *s_red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
    x = bc_comb(x, make_int2(__shfl_xor(x.x, o, 64), __shfl_xor(x.y, o, 64)));
  if ((threadIdx.x & (kWave - 1)) == 0) s_red[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kBcThreads / kWave; ++w) x = bc_comb(x, s_red[w]);
  __syncthreads();
  return x;
}

// Step 2 for heavy vertices: each item's extremes into A[pre(v)] by atomics
// (after k_bcc_local wrote the vertex's own), and step 4's rule for its
// non-tree edges.  Ends with a release as k_bcc_local.
template <class OffT>
__global__ __launch_bounds__(kBcThreads) void k_bcc_local_heavy(int64_t n, const OffT *__restrict__ off,
                                                                const int32_t *__restrict__ cols,
                                                                const int4 *__restrict__ R,
                                                                int2 *A, int32_t *L,
                                                                const int64_t *__restrict__ items,
                                                                int64_t item_cap,
                                                                const int32_t *__restrict__ counters) {
  __shared__ int2 s_red[kBcThreads / kWave];
  int64_t count = counters[kCntBccItems];
  if (count > item_cap) count = item_cap;
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    int64_t a0, a1;
    const int32_t u = (int32_t)bc_item(items, it, off, &a0, &a1);
    const int4 ru = R[u];
    int2 x = make_int2(INT32_MAX, INT32_MIN);
    for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
      const int32_t w = cols[a];
      if (w != u && w >= 0 && w < n && w != ru.x) {
        const int4 rw = R[w];
        if (rw.x != u) {
          x = bc_comb(x, make_int2(rw.y, rw.y));
          bc_cross(u, w, ru, rw, L);
        }
      }
    }
    x = bc_block_extremes(x, s_red);
    const int32_t pv = ru.y;
    if (threadIdx.x == 0 && pv >= 0 && pv < n && x.x <= x.y) {
      atomicMin(&reinterpret_cast<int *>(A)[2 * (int64_t)pv], x.x);
      atomicMax(&reinterpret_cast<int *>(A)[2 * (int64_t)pv + 1], x.y);
    }
  }
  block_release_device();
}

// Step 3a: one wave per block of 64 positions: prefix and suffix extremes
// within the block, and the block's extremes (level 0 of the sparse table).
__global__ __launch_bounds__(kBcThreads) void k_bcc_blocks(int64_t n, const int2 *__restrict__ A,
                                                           int2 *pfx, int2 *sfx, int2 *st0) {
  const int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int64_t nb = (n + kBcBlock - 1) / kBcBlock;
  if (b >= nb) return;   // a whole wave
  const int64_t i = b * kBcBlock + lane;
  const int2 x = i < n ? A[i] : make_int2(INT32_MAX, INT32_MIN);
  int2 f = x, s = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int2 u = make_int2(__shfl_up(f.x, o, 64), __shfl_up(f.y, o, 64));
    const int2 d = make_int2(__shfl_down(s.x, o, 64), __shfl_down(s.y, o, 64));
    if (lane >= o) f = bc_comb(f, u);
    if (lane + o < kWave) s = bc_comb(s, d);
  }
  if (i < n) {
    pfx[i] = f;
    sfx[i] = s;
  }
  if (lane == 0) st0[b] = s;
}

// Step 3b: level k of the sparse table over blocks (extremes of 2^k blocks).
__global__ __launch_bounds__(kBcThreads) void k_bcc_sparse(int64_t nb, int k, int2 *st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t h = (int64_t)1 << (k - 1);
  if (i + 2 * h > nb) return;
  st[k * nb + i] = bc_comb(st[(k - 1) * nb + i], st[(k - 1) * nb + i + h]);
}

// extremes of local over positions [l, r] (0 <= l <= r < n)
__device__ __forceinline__ int2 bc_range(int64_t l, int64_t r, const int2 *__restrict__ A,
                                         const int2 *__restrict__ pfx, const int2 *__restrict__ sfx,
                                         const int2 *__restrict__ st, int64_t nb) {
  const int64_t bl = l / kBcBlock, br = r / kBcBlock;
  if (bl == br) {
    if (l % kBcBlock == 0) return pfx[r];
    if (r % kBcBlock == kBcBlock - 1) return sfx[l];
    int2 m = A[l];
    for (int64_t i = l + 1; i <= r; ++i) m = bc_comb(m, A[i]);
    return m;
  }
  int2 m = bc_comb(sfx[l], pfx[r]);
  if (br - bl > 1) {
    const int64_t i = bl + 1, j = br - 1;
    const int k = 63 - __builtin_clzll((unsigned long long)(j - i + 1));
    m = bc_comb(m, st[k * nb + i]);
    m = bc_comb(m, st[k * nb + j - ((int64_t)1 << k) + 1]);
  }
  return m;
}

// every tree edge its own component to begin with (agent-scope stores: the
// hooking kernels after this one compare-and-swap these words)
template <int B>
__global__ __launch_bounds__(B) void k_bcc_iota(int64_t n, int32_t *L) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) store_agent(&L[v], (int32_t)v);
}

// Step 4, tree edges: v joins its parent's tree edge when a vertex of v's
// subtree reaches outside the parent's subtree.  Grid-stride over the
// vertices with a few workgroups per CU, each ending with one device-scope
// release (hooks in global memory, read on every XCD next): a release writes
// back the XCD's L2, and one per 256 vertices cost C4's pass as much as its
// gathers.
__global__ __launch_bounds__(kBcThreads) void k_bcc_rule_tree(int64_t n, const int4 *__restrict__ R,
                                                              const int2 *__restrict__ A,
                                                              const int2 *__restrict__ pfx,
                                                              const int2 *__restrict__ sfx,
                                                              const int2 *__restrict__ st, int64_t nb,
                                                              int32_t *L, int32_t *counters) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int4 a = R[v];
    const int32_t p = a.x;
    if (bc_is_root((int32_t)v, p, n)) continue;
    const int4 b = R[p];
    if (bc_is_root(p, b.x, n)) continue;
    const int64_t pv = a.y, sv = a.z, pp = b.y, sp = b.z;
    if (pv < 0 || sv < 1 || pv + sv > n || pp < 0 || sp < 1 || pp + sp > n) {
      atomicOr(&counters[kCntRangeErr], 1);
      continue;
    }
    const int2 lh = bc_range(pv, pv + sv - 1, A, pfx, sfx, st, nb);
    if (lh.x < pp || lh.y >= pp + sp) hook_join<true>((int32_t)v, p, L);
  }
  block_release_device();
}

// Step 5 setup: each vertex's final label into its record (R[x].w = L[x],
// L compressed).
__global__ __launch_bounds__(kBcThreads) void k_bcc_pack_labels(int64_t n, const int32_t *__restrict__ L,
                                                                int4 *R) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) reinterpret_cast<int32_t *>(R)[4 * x + 3] = L[x];
}

// The label of arc u -> w (u != w): its tree edge's when it is one (named by
// the child), else that of the tree edge of its later end in preorder.
__device__ __forceinline__ int32_t bc_arc_label(int32_t u, int32_t w, const int4 &ru,
                                                const int4 &rw) {
  if (rw.x == u) return rw.w;        // w is u's child
  if (ru.x == w) return ru.w;        // w is u's parent
  return ru.y > rw.y ? ru.w : rw.w;  // non-tree: the later end's tree edge
}

// Step 5 for heavy vertices: arc labels, and each vertex's label extremes into
// ext[v] (initialised by k_bcc_arcs) by atomics; k_bcc_art_heavy then decides
// the articulation points.
template <class OffT>
__global__ __launch_bounds__(kBcThreads) void k_bcc_arcs_heavy(int64_t n, const OffT *__restrict__ off,
                                                               const int32_t *__restrict__ cols,
                                                               const int4 *__restrict__ R,
                                                               int32_t *arc_label, int2 *ext,
                                                               const int64_t *__restrict__ items,
                                                               int64_t item_cap,
                                                               const int32_t *__restrict__ counters) {
  __shared__ int2 s_red[kBcThreads / kWave];
  int64_t count = counters[kCntBccItems];
  if (count > item_cap) count = item_cap;
  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    int64_t a0, a1;
    const int32_t u = (int32_t)bc_item(items, it, off, &a0, &a1);
    const int4 ru = R[u];
    int2 x = make_int2(INT32_MAX, -1);
    for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
      const int32_t w = cols[a];
      int32_t lab = -1;
      if (w != u && w >= 0 && w < n) {
        lab = bc_arc_label(u, w, ru, R[w]);
        x = bc_comb(x, make_int2(lab, lab));
      }
      arc_label[a] = lab;
    }
    x = bc_block_extremes(x, s_red);
    if (threadIdx.x == 0 && x.y >= 0) {
      atomicMin(&reinterpret_cast<int *>(ext)[2 * (int64_t)u], x.x);
      atomicMax(&reinterpret_cast<int *>(ext)[2 * (int64_t)u + 1], x.y);
    }
  }
}

__global__ __launch_bounds__(kBcThreads) void k_bcc_art_heavy(const int64_t *__restrict__ items,
                                                              int64_t item_cap, const int2 *__restrict__ ext,
                                                              uint8_t *art,
                                                              const int32_t *__restrict__ counters) {
  int64_t count = counters[kCntBccItems];
  if (count > item_cap) count = item_cap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < count; it += stride) {
    const int64_t item = items[it];
    if ((item & 0xffffffff) != 0) continue;   // once per vertex
    const int64_t v = item >> 32;
    const int2 e = ext[v];
    art[v] = (e.x != INT32_MAX && e.x != e.y) ? 1 : 0;
  }
}

// Sum of x over the workgroup added to *out by one atomic.  Called by all
// threads.
template <int B>
__device__ __forceinline__ void bc_block_add(int x, int32_t *out) {
  __shared__ int s_sum[B / kWave];
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if ((threadIdx.x & (kWave - 1)) == 0) s_sum[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < B / kWave; ++w) t += s_sum[w];
    if (t) atomicAdd(out, t);
  }
}

// Step 5: arc labels, articulation points, and the number of components
// (tree edges that are their component's smallest child), counted per
// workgroup: a tree whose edges are mostly bridges has about as many
// components as vertices, and an atomic per wave on the one counter
// serialised the pass (C4: 3.2 ms).
template <class OffT>
__global__ __launch_bounds__(kBcChunk, 8) void k_bcc_arcs(int64_t n, const OffT *__restrict__ off,
                                                       const int32_t *__restrict__ cols,
                                                       const int4 *__restrict__ R,
                                                       int32_t *arc_label, uint8_t *art,
                                                       int2 *ext, int32_t *counters) {
  __shared__ int s_scan[kBcChunk + 1];
  __shared__ OffT s_beg[kBcChunk];
  __shared__ int s_wave[kBcChunk / kWave];
  __shared__ int s_mn[kBcChunk], s_mx[kBcChunk];
  const int t = threadIdx.x;
  const int64_t chunks = (n + kBcChunk - 1) / kBcChunk;
  int comps = 0;
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int64_t v0 = c * kBcChunk, v = v0 + t;
    s_mn[t] = INT32_MAX;   // published by the scan's barriers
    s_mx[t] = -1;
    bc_chunk_arcs(n, v0, off, cols, s_scan, s_beg, s_wave,
                  [&](int j, int32_t u, int32_t w, int64_t a) {
                    int32_t lab = -1;
                    int2 val = make_int2(INT32_MAX, -1);
                    if (j >= 0 && w != u && w >= 0 && w < n) {
                      lab = bc_arc_label(u, w, R[u], R[w]);
                      val = make_int2(lab, lab);
                    }
                    if (j >= 0) arc_label[a] = lab;
                    bc_run_extremes(j, val, s_mn, s_mx);
                  });
    if (v < n) {
      // a heavy vertex's arcs are the item pass's; its extremes start from
      // its own chunk's (none)
      if ((int64_t)(off[v + 1] - off[v]) > kBcHeavy) ext[v] = make_int2(s_mn[t], s_mx[t]);
      if (art) art[v] = (s_mn[t] != INT32_MAX && s_mn[t] != s_mx[t]) ? 1 : 0;
      const int4 rv = R[v];
      comps += !bc_is_root((int32_t)v, rv.x, n) && rv.w == (int32_t)v;
    }
  }
  bc_block_add<kBcChunk>(comps, &counters[kCntComponents]);
}

static unsigned bc_grid(const rst_ctx *ctx, int64_t n) {
  const int64_t chunks = (n + kBcChunk - 1) / kBcChunk;
  const int64_t cap = (int64_t)ctx->num_cus * 2;
  return (unsigned)(chunks < cap ? (chunks < 1 ? 1 : chunks) : cap);
}

template <class OffT>
static rst_status bc_arc_passes(rst_ctx *ctx, const rst_csr *g, int4 *R, int2 *A, int2 *pfx,
                                int2 *sfx, int2 *st, int64_t nb, int levels, int32_t *L,
                                int64_t *items, int64_t item_cap, int32_t *arc_label, uint8_t *art,
                                int32_t *counters) {
  const int64_t n = g->n;
  const OffT *off = static_cast<const OffT *>(g->offsets);
  const unsigned grid = bc_grid(ctx, n);
  const unsigned hgrid = (unsigned)(ctx->num_cus * 4);
  RST_SWEEP(ctx, k_bcc_iota, n, n, L);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bcc_local<OffT>, dim3(grid), dim3(kBcChunk), 0, ctx->stream, n, off, g->cols,
                     R, A, L, items, item_cap, counters);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bcc_local_heavy<OffT>, dim3(hgrid), dim3(kBcThreads), 0, ctx->stream, n, off,
                     g->cols, R, A, L, items, item_cap, counters);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bcc_blocks, dim3(grid_for(nb * kWave, kBcThreads)), dim3(kBcThreads), 0,
                     ctx->stream, n, A, pfx, sfx, st);
  RST_HIP(hipGetLastError());
  for (int k = 1; k < levels; ++k) {
    hipLaunchKernelGGL(k_bcc_sparse, dim3(grid_for(nb, kBcThreads)), dim3(kBcThreads), 0,
                       ctx->stream, nb, k, st);
    RST_HIP(hipGetLastError());
  }
  const int64_t tblocks = (n + kBcThreads - 1) / kBcThreads;
  const unsigned tgrid = (unsigned)(tblocks < ctx->num_cus * 8 ? tblocks : ctx->num_cus * 8);
  hipLaunchKernelGGL(k_bcc_rule_tree, dim3(tgrid), dim3(kBcThreads), 0, ctx->stream, n, R, A, pfx,
                     sfx, st, nb, L, counters);
  RST_HIP(hipGetLastError());
  RST_TRY(enqueue_compress(ctx, n, L, nullptr, nullptr));
  hipLaunchKernelGGL(k_bcc_pack_labels, dim3(grid_for(n, kBcThreads)), dim3(kBcThreads), 0,
                     ctx->stream, n, L, R);
  RST_HIP(hipGetLastError());
  // the range structure is done with: pfx holds each heavy vertex's label
  // extremes from here on (indexed by vertex)
  int2 *ext = pfx;
  hipLaunchKernelGGL(k_bcc_arcs<OffT>, dim3(grid), dim3(kBcChunk), 0, ctx->stream, n, off, g->cols,
                     R, arc_label, art, ext, counters);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bcc_arcs_heavy<OffT>, dim3(hgrid), dim3(kBcThreads), 0, ctx->stream, n, off,
                     g->cols, R, arc_label, ext, items, item_cap, counters);
  RST_HIP(hipGetLastError());
  if (art) {
    hipLaunchKernelGGL(k_bcc_art_heavy, dim3(grid_for(item_cap, kBcThreads)), dim3(kBcThreads), 0,
                       ctx->stream, items, item_cap, ext, art, counters);
    RST_HIP(hipGetLastError());
  }
  return RST_OK;
}

rst_status run_biconnected(rst_ctx *ctx, const rst_csr *g, const int32_t *parent,
                           int32_t *arc_label, uint8_t *art, int64_t *num_components) {
  const int64_t n = g->n;
  const GlistPlan plan = glist_plan(2 * n, n / 2 + 1, ctx->opt.rank_stride);
  const int64_t nb = (n + kBcBlock - 1) / kBcBlock;
  int levels = 1;   // floor(log2 nb) + 1
  while (((int64_t)1 << levels) <= nb) ++levels;
  // heavy items: every heavy vertex has more than kBcHeavy arcs
  const int64_t item_cap = g->nnz / kBcHeavy + g->nnz / kBcSlice + 1;
  RST_TRY(ws_reserve(ctx, depth_ws_bytes(n, plan) + ws_bytes((size_t)n, 16) +
                              ws_bytes((size_t)n, 4) + 3 * ws_bytes((size_t)n, 8) +
                              ws_bytes((size_t)(levels * nb), 8) + ws_bytes((size_t)item_cap, 8)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  // per vertex (parent, pre, nd, label): one gather for all that an arc pass
  // needs of its far end
  int4 *R = ws_take<int4>(ctx, n);
  int32_t *L = ws_take<int32_t>(ctx, n);
  int2 *A = ws_take<int2>(ctx, n);
  int2 *pfx = ws_take<int2>(ctx, n);
  int2 *sfx = ws_take<int2>(ctx, n);
  int2 *st = ws_take<int2>(ctx, (size_t)(levels * nb));
  int64_t *items = ws_take<int64_t>(ctx, (size_t)item_cap);
  RST_TRY(enqueue_fill(ctx, counters, 32, 0));
  RST_TRY(run_tour_preorder(ctx, n, parent, R, counters));
  if (ctx->host_pinned[kCntBccRoots] != 1) return RST_E_DISCONNECTED;
  if (g->offset_bytes == 4)
    RST_TRY(bc_arc_passes<int32_t>(ctx, g, R, A, pfx, sfx, st, nb, levels, L, items, item_cap,
                                   arc_label, art, counters));
  else
    RST_TRY(bc_arc_passes<int64_t>(ctx, g, R, A, pfx, sfx, st, nb, levels, L, items, item_cap,
                                   arc_label, art, counters));
  RST_HIP(hipMemcpyAsync(ctx->host_pinned, counters, kCntTotal * sizeof(int32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->host_pinned[kCntRangeErr]) return RST_E_RANGE;
  if (num_components) *num_components = ctx->host_pinned[kCntComponents];
  return RST_OK;
}

}  // namespace rst

using namespace rst;

extern "C" rst_status rst_biconnected(rst_ctx *ctx, const rst_csr *g, const int32_t *parent,
                                      int32_t *arc_label, uint8_t *articulation,
                                      int64_t *num_components) {
  if (!ctx || !g || !parent || g->n < 1 || !g->offsets) return RST_E_INVAL;
  if (g->nnz < 0 || (g->nnz > 0 && (!g->cols || !arc_label))) return RST_E_INVAL;
  if (g->offset_bytes != 4 && g->offset_bytes != 8) return RST_E_INVAL;
  // arc ids of the tour (2n) and the per-workgroup arc counts are int32
  if (g->n >= ((int64_t)1 << 30) || g->nnz >= ((int64_t)1 << 31)) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  return run_biconnected(ctx, g, parent, arc_label, articulation, num_components);
}
