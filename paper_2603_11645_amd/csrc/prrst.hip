// prrst.hip -- Path-Reversal RST (Sec. III-C, after Cong and Bader).
//
// A rooted spanning forest P is kept at all times (every vertex its own root
// at the start).  One iteration:
//  1. special ancestors by pointer jumping: anc[0] = P, anc[k+1][v] =
//     anc[k][anc[k][v]]; a level that changes nothing ends the jumping (every
//     pointer of the level before already reaches its root), and the last
//     level computed gives every vertex's representative (its root);
//  2. hooking, alternating max and min representatives: for an edge (u, w)
//     joining two trees, the tree of the smaller representative (max round)
//     or of the larger (min round) is grafted; its root r records the edge
//     as (x in r's tree, y in the other) with one 64-bit store (any edge
//     may win; a pair is never torn);
//  3. path marking: x of every grafted root is marked, then in round k every
//     marked vertex marks its 2^k-th ancestor, over the levels computed in 1
//     (every marked vertex is an ancestor of x, so marking within a round is
//     harmless and the rounds reach the root);
//  4. reversal and graft: for every marked non-root v, P'[P[v]] = v, and
//     P'[x] = y for every grafted root, into a second parent array.
// The loop ends when no edge joins two trees.  Finally the tree of the
// designated root, and every other tree at its minimum id, is re-rooted by
// the same marking and reversal.  The host synchronises once per iteration
// (the hook flag); the paper's GPU version takes several pointer-jumping
// steps per synchronisation, here every level of the jumping is one launch
// and the launches run back to back.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

constexpr int kPrThreads = 1024;
constexpr uint64_t kPrNoHook = ~0ull;

__global__ __launch_bounds__(kBlock) void k_pr_iota(int64_t n, int32_t *p) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) p[v] = (int32_t)v;
}

// anc[k+1] from anc[k] unless level k-1 changed nothing (then anc[k] is final
// and this level is not computed).  changed: int32 [levels] flags.
__global__ __launch_bounds__(kBlock) void k_pr_jump(int64_t n, int k, const int32_t *__restrict__ src,
                                                    int32_t *dst, int32_t *changed) {
  if (k > 0 && !changed[k - 1]) return;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (v < n) {
    const int32_t a = src[v];
    const int32_t b = src[a];
    dst[v] = b;
    ch = b != a;
  }
  if (__ballot(ch) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&changed[k], 1);
}

// the last level computed: anc[top] holds every vertex's root
__device__ __forceinline__ int pr_top(const int32_t *changed, int levels) {
  int k = 0;
  while (k < levels - 1 && changed[k]) ++k;
  return k;
}

// Hooking over all arcs (u, w) with u < w, edge-centric: a workgroup takes
// 1024 consecutive vertices, scans their degrees in LDS and walks the union
// of their arcs with unit stride.
template <class OffT>
__global__ __launch_bounds__(kPrThreads) void k_pr_hook(int64_t n, const OffT *__restrict__ off,
                                                        const int32_t *__restrict__ cols,
                                                        const int32_t *__restrict__ anc, int levels,
                                                        const int32_t *__restrict__ changed,
                                                        int max_round, uint64_t *win,
                                                        int32_t *counters) {
  __shared__ int s_scan[kPrThreads + 1];
  __shared__ OffT s_beg[kPrThreads];
  __shared__ int s_wave[kPrThreads / kWave];
  const int top = pr_top(changed, levels);
  const int32_t *rep = anc + (size_t)top * (size_t)n;
  const int t = threadIdx.x;
  const int64_t v = (int64_t)blockIdx.x * kPrThreads + t;
  int deg = 0;
  OffT beg = 0;
  if (v < n) {
    beg = off[v];
    deg = (int)(off[v + 1] - beg);
  }
  s_beg[t] = beg;
  int total;
  const int excl = block_excl_scan<kPrThreads>(deg, s_wave, &total);
  s_scan[t] = excl;
  if (t == kPrThreads - 1) s_scan[kPrThreads] = excl + deg;
  __syncthreads();
  const int64_t v0 = (int64_t)blockIdx.x * kPrThreads;
  bool any = false;
  for (int b = 0; b < total; b += kPrThreads) {
    const int k = b + t;
    if (k < total) {
      const int j = lds_upper_search(s_scan, kPrThreads, k);
      const int32_t u = (int32_t)(v0 + j);
      const int32_t w = cols[(int64_t)s_beg[j] + (k - s_scan[j])];
      if (u < w) {
        const int32_t ru = rep[u], rw = rep[w];
        if (ru != rw) {
          const bool u_grafted = max_round ? ru < rw : ru > rw;
          const int32_t r = u_grafted ? ru : rw;
          const int32_t x = u_grafted ? u : w, y = u_grafted ? w : u;
          win[r] = ((uint64_t)(uint32_t)y << 32) | (uint32_t)x;
          any = true;
        }
      }
    }
  }
  if (__ballot(any) != 0ull && (t & 63) == 0) atomicOr(&counters[kCntPrHooks], 1);
}

// on[x] = 1 for every grafted root's x
__global__ __launch_bounds__(kBlock) void k_pr_mark_start(int64_t n, const uint64_t *__restrict__ win,
                                                          uint8_t *on) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint64_t wv = win[r];
  if (wv != kPrNoHook) on[(int32_t)(uint32_t)wv] = 1;
}

// one marking round: every marked vertex marks its 2^k-th ancestor
__global__ __launch_bounds__(kBlock) void k_pr_mark(int64_t n, int k, const int32_t *__restrict__ anck,
                                                    const int32_t *__restrict__ changed, int levels,
                                                    uint8_t *on) {
  if (k > pr_top(changed, levels)) return;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && on[v]) on[anck[v]] = 1;
}

// P2 = P beforehand; reversal along marked paths, then the grafts
__global__ __launch_bounds__(kBlock) void k_pr_reverse(int64_t n, const int32_t *__restrict__ P,
                                                       int32_t *P2, const uint8_t *__restrict__ on,
                                                       const uint64_t *__restrict__ win) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t p = P[v];
  if (on[v] && p != (int32_t)v) P2[p] = (int32_t)v;
  if (win) {
    const uint64_t wv = win[v];
    if (wv != kPrNoHook) P2[(int32_t)(uint32_t)wv] = (int32_t)(wv >> 32);
  }
}

// Final re-rooting targets: min id of every tree (atomic minimum over its
// vertices, skipped where the minimum read beforehand is already smaller:
// in one large tree every vertex's atomic would go to the same word) ...
__global__ __launch_bounds__(kBlock) void k_pr_minid(int64_t n, const int32_t *__restrict__ anc,
                                                     int levels, const int32_t *__restrict__ changed,
                                                     int32_t *minid) {
  const int32_t *rep = anc + (size_t)pr_top(changed, levels) * (size_t)n;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    int32_t *m = &minid[rep[v]];
    if ((int32_t)v < __hip_atomic_load(m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMin(m, (int32_t)v);
  }
}

// ... then on[t] = 1 for the designated root and for the minimum id of every
// tree that does not hold it; trees are counted.
__global__ __launch_bounds__(kBlock) void k_pr_targets(int64_t n, const int32_t *__restrict__ anc,
                                                       int levels,
                                                       const int32_t *__restrict__ changed,
                                                       const int32_t *__restrict__ minid,
                                                       const int32_t *__restrict__ rootbuf,
                                                       uint8_t *on, int32_t *counters) {
  const int32_t *rep = anc + (size_t)pr_top(changed, levels) * (size_t)n;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t R = rootbuf[0];
  bool tree = false;
  if (v < n && rep[v] == (int32_t)v) {
    tree = true;
    on[v == rep[R] ? R : minid[v]] = 1;
  }
  wave_count(tree, &counters[kCntComponents]);
}

// P2 = P with every target t made a root
__global__ __launch_bounds__(kBlock) void k_pr_set_roots(int64_t n, const uint8_t *__restrict__ target,
                                                         int32_t *P2) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && target[v]) P2[v] = (int32_t)v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static int pr_levels(int64_t n) {
  int k = 1;
  while (((int64_t)1 << (k - 1)) < n) ++k;
  return k;   // 2^(levels-1) >= n: anc[levels-1] reaches every root
}

size_t prrst_ws_bytes(int64_t n) {
  const int L = pr_levels(n);
  return ws_bytes(64, 4) + (size_t)(L + 2) * ws_bytes((size_t)n, 4) + 2 * ws_bytes((size_t)n, 1) +
         ws_bytes((size_t)n, 8) + ws_bytes(64, 4);
}

// the jumping levels of the forest in P into anc (anc[0] = P copied)
static rst_status pr_jumps(rst_ctx *ctx, int64_t n, const int32_t *P, int32_t *anc, int levels,
                           int32_t *changed) {
  RST_TRY(enqueue_fill(ctx, changed, levels, 0));
  RST_HIP(hipMemcpyAsync(anc, P, (size_t)n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  for (int k = 0; k + 1 < levels; ++k) {
    hipLaunchKernelGGL(k_pr_jump, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, k,
                       anc + (size_t)k * (size_t)n, anc + (size_t)(k + 1) * (size_t)n, changed);
    RST_HIP(hipGetLastError());
  }
  return RST_OK;
}

static rst_status pr_marks(rst_ctx *ctx, int64_t n, const int32_t *anc, int levels,
                           const int32_t *changed, uint8_t *on) {
  for (int k = 0; k < levels; ++k) {
    hipLaunchKernelGGL(k_pr_mark, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, k,
                       anc + (size_t)k * (size_t)n, changed, levels, on);
    RST_HIP(hipGetLastError());
  }
  return RST_OK;
}

rst_status run_pr_rst(rst_ctx *ctx, const rst_csr *g, int32_t root, int32_t *parent,
                      int64_t *iterations, int64_t *components) {
  const int64_t n = g->n;
  const int levels = pr_levels(n);
  RST_TRY(ws_reserve(ctx, prrst_ws_bytes(n)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  int32_t *rootbuf = counters + 32;
  int32_t *anc = ws_take<int32_t>(ctx, (size_t)levels * (size_t)n);
  int32_t *P2 = ws_take<int32_t>(ctx, n);
  int32_t *minid = ws_take<int32_t>(ctx, n);
  uint8_t *on = ws_take<uint8_t>(ctx, n);
  uint8_t *target = ws_take<uint8_t>(ctx, n);
  uint64_t *win = ws_take<uint64_t>(ctx, n);
  int32_t *changed = ws_take<int32_t>(ctx, 64);
  RST_TRY(enqueue_reset_counters(ctx, counters, root));
  int32_t *P = parent;
  hipLaunchKernelGGL(k_pr_iota, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, P);
  RST_HIP(hipGetLastError());
  const unsigned hook_grid = grid_for(n, kPrThreads);
  int64_t it = 0;
  for (;; ++it) {
    if (it > 4 * n + 64) return RST_E_DEVICE;   // cannot happen: the forest shrinks
    RST_TRY(pr_jumps(ctx, n, P, anc, levels, changed));
    RST_TRY(enqueue_fill(ctx, reinterpret_cast<int32_t *>(win), 2 * n, -1));
    RST_TRY(enqueue_fill(ctx, counters + kCntPrHooks, 1, 0));
    if (g->offset_bytes == 4)
      hipLaunchKernelGGL(k_pr_hook<int32_t>, dim3(hook_grid), dim3(kPrThreads), 0, ctx->stream, n,
                         (const int32_t *)g->offsets, g->cols, anc, levels, changed,
                         (int)((it & 1) == 0), win, counters);
    else
      hipLaunchKernelGGL(k_pr_hook<int64_t>, dim3(hook_grid), dim3(kPrThreads), 0, ctx->stream, n,
                         (const int64_t *)g->offsets, g->cols, anc, levels, changed,
                         (int)((it & 1) == 0), win, counters);
    RST_HIP(hipGetLastError());
    RST_HIP(hipMemcpyAsync(ctx->host_pinned, counters + kCntPrHooks, sizeof(int32_t),
                           hipMemcpyDeviceToHost, ctx->stream));
    RST_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->host_pinned[0] == 0) break;
    RST_TRY(enqueue_fill(ctx, reinterpret_cast<int32_t *>(on), (n + 3) / 4, 0));
    hipLaunchKernelGGL(k_pr_mark_start, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n,
                       win, on);
    RST_HIP(hipGetLastError());
    RST_TRY(pr_marks(ctx, n, anc, levels, changed, on));
    RST_HIP(hipMemcpyAsync(P2, P, (size_t)n * 4, hipMemcpyDeviceToDevice, ctx->stream));
    hipLaunchKernelGGL(k_pr_reverse, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, P,
                       P2, on, win);
    RST_HIP(hipGetLastError());
    std::swap(P, P2);
  }
  // re-root: the designated root's tree at it, every other tree at its minimum id
  RST_TRY(enqueue_fill(ctx, minid, n, 0x7fffffff));
  RST_TRY(enqueue_fill(ctx, reinterpret_cast<int32_t *>(on), (n + 3) / 4, 0));
  RST_TRY(enqueue_fill(ctx, counters + kCntComponents, 1, 0));
  // the special ancestors of the final forest are those of the last
  // iteration's jumping (no hook since)
  hipLaunchKernelGGL(k_pr_minid, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, anc,
                     levels, changed, minid);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pr_targets, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, anc,
                     levels, changed, minid, rootbuf, on, counters);
  RST_HIP(hipGetLastError());
  RST_HIP(hipMemcpyAsync(target, on, (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
  RST_TRY(pr_marks(ctx, n, anc, levels, changed, on));
  RST_HIP(hipMemcpyAsync(P2, P, (size_t)n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  hipLaunchKernelGGL(k_pr_reverse, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, P,
                     P2, on, nullptr);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pr_set_roots, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n,
                     target, P2);
  RST_HIP(hipGetLastError());
  if (P2 != parent)
    RST_HIP(hipMemcpyAsync(parent, P2, (size_t)n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  RST_HIP(hipMemcpyAsync(ctx->host_pinned, counters, kCntTotal * sizeof(int32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->host_pinned[kCntRangeErr]) return RST_E_INVAL;
  if (iterations) *iterations = it;
  if (components) *components = ctx->host_pinned[kCntComponents];
  return RST_OK;
}

}  // namespace rst
