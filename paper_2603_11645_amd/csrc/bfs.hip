// bfs.hip -- level-synchronous breadth-first search (Sec. III-A), the baseline.
//
// Each level is one kernel launch over the current frontier: every frontier
// vertex offers all its arcs, an unvisited neighbour is claimed with a
// compare-and-swap on its level (the winner's source becomes its parent) and
// appended to the next frontier.  Load balance follows the edge-centric idea of
// Merrill et al. (Sec. II): a block takes 256 frontier vertices, scans their
// degrees in LDS and walks the union of their arcs with unit stride, so a
// thread handles arcs, not vertices.  Vertices above a degree threshold go to
// a separate "heavy" frontier whose arcs are split across all blocks.
// Appends use one atomic per wavefront (ballot + mbcnt).
//
// Frontier sizes live in device memory, so the host enqueues several levels
// back to back and only reads the frontier size once per batch; a level whose
// input frontier is empty returns at once.  Counts rotate over three slots:
// level L reads slot L%3, appends to slot (L+1)%3 and clears slot (L+2)%3,
// which the next launch appends to.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

__global__ void k_bfs_reset(int64_t n, int32_t *level, int32_t *parent, int32_t *cnt) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    level[v] = -1;
    if (parent) parent[v] = -1;
  }
  if (v < 6) cnt[v] = 0;
}

template <class OffT>
__device__ __forceinline__ void bfs_enqueue(bool win, int32_t w, const OffT *off, int heavy_deg,
                                            int32_t *qout, int32_t *hout, int32_t *cout,
                                            int64_t heavy_cap, int32_t *counters) {
  bool heavy = false;
  if (win) heavy = (int64_t)(off[w + 1] - off[w]) > heavy_deg;
  const bool light = win && !heavy;
  const int sl = wave_append(light, &cout[0]);
  if (light) qout[sl] = w;
  const int sh = wave_append(win && heavy, &cout[1]);
  if (win && heavy && sh < heavy_cap) hout[sh] = w;
  wave_count(win, &counters[kCntBfsReached]);
}

template <class OffT>
__global__ __launch_bounds__(kBlock) void k_bfs_seed(const int32_t *__restrict__ roots,
                                                     int32_t nroots, int64_t n,
                                                     const OffT *__restrict__ off, int32_t *level,
                                                     int32_t *parent, int32_t *q0, int32_t *h0,
                                                     int32_t *cnt0, int64_t heavy_cap,
                                                     int32_t *counters, int heavy_deg,
                                                     const uint8_t *__restrict__ gsel) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t r = -1;
  bool win = false;
  if (i < nroots && (!gsel || gsel[i])) {
    r = roots[i];
    if (r < 0 || r >= n) atomicOr(&counters[kCntRangeErr], 1);
    else if (atomicCAS(&level[r], -1, 0) == -1) {
      win = true;
      if (parent) parent[r] = r;
    }
  }
  bfs_enqueue<OffT>(win, r, off, heavy_deg, q0, h0, cnt0, heavy_cap, counters);
}

template <class OffT>
__global__ __launch_bounds__(kBlock) void k_bfs_seed_unreached(int64_t n, const OffT *__restrict__ off,
                                                               const int32_t *__restrict__ cc,
                                                               int32_t *level, int32_t *parent,
                                                               int32_t *q0, int32_t *h0, int32_t *cnt0,
                                                               int64_t heavy_cap, int32_t *counters,
                                                               int heavy_deg,
                                                               const uint8_t *__restrict__ vsel) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool win = false;
  if (v < n && cc[v] == (int32_t)v && level[v] == -1 && (!vsel || vsel[v])) {
    level[v] = 0;
    parent[v] = (int32_t)v;
    win = true;
  }
  bfs_enqueue<OffT>(win, (int32_t)v, off, heavy_deg, q0, h0, cnt0, heavy_cap, counters);
}

template <class OffT>
__global__ __launch_bounds__(kBlock) void k_bfs_level(
    int32_t L, const OffT *__restrict__ off, const int32_t *__restrict__ cols, int32_t *level,
    int32_t *parent, const int32_t *__restrict__ qin, const int32_t *__restrict__ hin,
    const int32_t *cin, int32_t *qout, int32_t *hout, int32_t *cout, int32_t *czero,
    int64_t heavy_cap, int32_t *counters, int heavy_deg) {
  __shared__ int s_scan[kBlock + 1];
  __shared__ OffT s_beg[kBlock];
  __shared__ int32_t s_src[kBlock];
  __shared__ int s_wave[kBlock / kWave];
  const int nl = cin[0];
  int nh = cin[1];
  if (nh > heavy_cap) nh = (int)heavy_cap;
  if (blockIdx.x == 0 && threadIdx.x < 2) czero[threadIdx.x] = 0;
  if (nl + nh == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) counters[kCntBfsLast] = L;
  const int t = threadIdx.x;
  const int32_t next_level = L + 1;

  for (int64_t c0 = (int64_t)blockIdx.x * kBlock; c0 < nl; c0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = c0 + t;
    int deg = 0;
    OffT beg = 0;
    int32_t u = -1;
    if (i < nl) {
      u = qin[i];
      beg = off[u];
      deg = (int)(off[u + 1] - beg);
    }
    s_beg[t] = beg;
    s_src[t] = u;
    int total;
    const int excl = block_excl_scan<kBlock>(deg, s_wave, &total);
    s_scan[t] = excl;
    if (t == kBlock - 1) s_scan[kBlock] = excl + deg;
    __syncthreads();
    for (int b = 0; b < total; b += kBlock) {
      const int k = b + t;
      int32_t w = -1, src = -1;
      if (k < total) {
        const int j = lds_upper_search(s_scan, kBlock, k);
        src = s_src[j];
        w = cols[(int64_t)s_beg[j] + (k - s_scan[j])];
      }
      bool win = false;
      if (w >= 0 && level[w] == -1 && atomicCAS(&level[w], -1, next_level) == -1) {
        win = true;
        if (parent) parent[w] = src;
      }
      bfs_enqueue<OffT>(win, w, off, heavy_deg, qout, hout, cout, heavy_cap, counters);
    }
    __syncthreads();
  }

  for (int hi = 0; hi < nh; ++hi) {
    const int32_t u = hin[hi];
    const int64_t b = (int64_t)off[u], e = (int64_t)off[u + 1];
    for (int64_t a0 = b + (int64_t)blockIdx.x * kBlock; a0 < e; a0 += (int64_t)gridDim.x * kBlock) {
      const int64_t a = a0 + t;
      const int32_t w = a < e ? cols[a] : -1;
      bool win = false;
      if (w >= 0 && level[w] == -1 && atomicCAS(&level[w], -1, next_level) == -1) {
        win = true;
        if (parent) parent[w] = u;
      }
      bfs_enqueue<OffT>(win, w, off, heavy_deg, qout, hout, cout, heavy_cap, counters);
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

size_t bfs_heavy_capacity(const rst_ctx *ctx, int64_t n, int64_t nnz) {
  const int64_t heavy = ctx->opt.bfs_heavy_degree < 1 ? 1 : ctx->opt.bfs_heavy_degree;
  int64_t cap = nnz / (heavy + 1) + 1;
  return (size_t)(cap < n ? cap : n);
}

rst_status bfs_reset(rst_ctx *ctx, int64_t n, int32_t *level, int32_t *parent, BfsBufs &b) {
  const int64_t items = n > 6 ? n : 6;
  hipLaunchKernelGGL(k_bfs_reset, dim3(grid_for(items, kBlock)), dim3(kBlock), 0, ctx->stream, n,
                     level, parent, b.cnt);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status bfs_seed_roots(rst_ctx *ctx, const rst_csr *g, const int32_t *roots, int32_t nroots,
                          int32_t *level, int32_t *parent, BfsBufs &b, int32_t *counters,
                          const uint8_t *gsel) {
  const int hd = ctx->opt.bfs_heavy_degree;
  if (g->offset_bytes == 4)
    hipLaunchKernelGGL(k_bfs_seed<int32_t>, dim3(grid_for(nroots, kBlock)), dim3(kBlock), 0,
                       ctx->stream, roots, nroots, g->n, (const int32_t *)g->offsets, level, parent,
                       b.q[0], b.h[0], b.cnt, b.heavy_cap, counters, hd, gsel);
  else
    hipLaunchKernelGGL(k_bfs_seed<int64_t>, dim3(grid_for(nroots, kBlock)), dim3(kBlock), 0,
                       ctx->stream, roots, nroots, g->n, (const int64_t *)g->offsets, level, parent,
                       b.q[0], b.h[0], b.cnt, b.heavy_cap, counters, hd, gsel);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status bfs_seed_unreached(rst_ctx *ctx, const rst_csr *g, const int32_t *cc, int32_t *level,
                              int32_t *parent, BfsBufs &b, int32_t *counters,
                              const uint8_t *vsel) {
  const int hd = ctx->opt.bfs_heavy_degree;
  // counts of slot 0 must start from zero for this new frontier
  RST_TRY(enqueue_fill(ctx, b.cnt, 6, 0));
  if (g->offset_bytes == 4)
    hipLaunchKernelGGL(k_bfs_seed_unreached<int32_t>, dim3(grid_for(g->n, kBlock)), dim3(kBlock), 0,
                       ctx->stream, g->n, (const int32_t *)g->offsets, cc, level, parent, b.q[0],
                       b.h[0], b.cnt, b.heavy_cap, counters, hd, vsel);
  else
    hipLaunchKernelGGL(k_bfs_seed_unreached<int64_t>, dim3(grid_for(g->n, kBlock)), dim3(kBlock), 0,
                       ctx->stream, g->n, (const int64_t *)g->offsets, cc, level, parent, b.q[0],
                       b.h[0], b.cnt, b.heavy_cap, counters, hd, vsel);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

template <class OffT>
static rst_status launch_level(rst_ctx *ctx, const rst_csr *g, int32_t L, unsigned grid,
                               int32_t *level, int32_t *parent, BfsBufs &b, int32_t *counters) {
  const int cur = L % 3, nxt = (L + 1) % 3, clr = (L + 2) % 3;
  hipLaunchKernelGGL(k_bfs_level<OffT>, dim3(grid), dim3(kBlock), 0, ctx->stream, L,
                     (const OffT *)g->offsets, g->cols, level, parent, b.q[L & 1], b.h[L & 1],
                     b.cnt + 2 * cur, b.q[(L + 1) & 1], b.h[(L + 1) & 1], b.cnt + 2 * nxt,
                     b.cnt + 2 * clr, b.heavy_cap, counters, ctx->opt.bfs_heavy_degree);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status bfs_run_levels(rst_ctx *ctx, const rst_csr *g, int32_t *level, int32_t *parent,
                          BfsBufs &b, int32_t *counters, int64_t *levels_out, int64_t max_levels) {
  const int per_sync = ctx->opt.bfs_levels_per_sync < 1 ? 1 : ctx->opt.bfs_levels_per_sync;
  const unsigned grid = ctx->opt.bfs_grid > 0 ? (unsigned)ctx->opt.bfs_grid
                                              : (unsigned)(ctx->num_cus * 4);
  int64_t L = 0;
  for (;;) {
    for (int k = 0; k < per_sync && (max_levels < 0 || L < max_levels); ++k, ++L) {
      if (g->offset_bytes == 4)
        RST_TRY(launch_level<int32_t>(ctx, g, (int32_t)L, grid, level, parent, b, counters));
      else
        RST_TRY(launch_level<int64_t>(ctx, g, (int32_t)L, grid, level, parent, b, counters));
    }
    // frontier feeding level L (written by level L-1)
    RST_HIP(hipMemcpyAsync(ctx->host_pinned, b.cnt + 2 * (L % 3), 2 * sizeof(int32_t),
                           hipMemcpyDeviceToHost, ctx->stream));
    RST_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->host_pinned[0] == 0 && ctx->host_pinned[1] == 0) break;
    if (max_levels >= 0 && L >= max_levels) break;   // capped search (depth probes)
    if (L > g->n + per_sync) return RST_E_DEVICE;   // cannot happen for a valid CSR
  }
  RST_HIP(hipMemcpyAsync(ctx->host_pinned + 2, counters + kCntBfsLast, sizeof(int32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  if (levels_out) *levels_out = ctx->host_pinned[2];
  return RST_OK;
}

}  // namespace rst
