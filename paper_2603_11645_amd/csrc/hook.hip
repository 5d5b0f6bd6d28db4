// hook.hip -- connectivity with spanning-edge recording (Sec. III-B, Sec. I).
//
// Hooking: for an undirected edge (u,v) whose endpoints lie in different
// trees, the larger of the two tree roots is linked under the smaller one by a
// compare-and-swap that only succeeds on a root (hooking by vertex id).  The
// edge behind every successful hook is stored at the root that was hooked
// (tu[hi], tv[hi]), so the n - c non-roots carry exactly the edges of a
// spanning forest.  Root finding uses path halving, i.e. the pointer-jumping
// step P[i] = P[P[i]] applied along the search path, so hooking and compression
// are interleaved in one asynchronous sweep; a final pass (compress) points
// every vertex at its root, which is the minimum id of its component because
// every pointer goes from a larger id to a smaller one.
//
// Work split (MI355X): a block of 256 threads owns 256 consecutive vertices,
// stages their arc ranges in LDS with a block scan and walks the union of their
// arcs with unit stride, so cols[] is read coalesced.  A vertex of degree
// above a threshold is not expanded by its block; its arcs are cut into fixed
// chunks and handed to a second launch that spreads them over the whole grid,
// so a 10^5-degree hub cannot serialise one block.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

constexpr int kChunk = 4096;   // arcs per heavy-vertex chunk

// ---------------------------------------------------------------------------
// union-find core
// ---------------------------------------------------------------------------

// Root of x with path halving.  Invariant cc[y] <= y (equality iff y is a root)
// makes the walk strictly decreasing, so it ends even on stale reads; the plain
// stores only ever replace a non-root's pointer by one of its ancestors.
__device__ __forceinline__ int32_t find_root(int32_t x, int32_t *cc) {
  int32_t cur = cc[x];
  if (cur != x) {
    int32_t prev = x, nxt;
    while (cur > (nxt = cc[cur])) {
      cc[prev] = nxt;
      prev = cur;
      cur = nxt;
    }
  }
  return cur;
}

// Hook the trees of u and v; on success record (u,v) at the hooked root.
template <bool kRecord>
__device__ __forceinline__ void hook_edge(int32_t u, int32_t v, int32_t *cc, int32_t *tu,
                                          int32_t *tv) {
  int32_t ru = find_root(u, cc);
  int32_t rv = find_root(v, cc);
  while (ru != rv) {
    const int32_t lo = ru < rv ? ru : rv;
    const int32_t hi = ru < rv ? rv : ru;
    const int32_t old = atomicCAS(&cc[hi], hi, lo);
    if (old == hi) {
      if (kRecord) { tu[hi] = u; tv[hi] = v; }
      return;
    }
    // hi was hooked meanwhile: continue from its new parent (an ancestor)
    if (ru == hi) ru = old; else rv = old;
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

template <class OffT>
__global__ __launch_bounds__(kBlock) void k_validate(int64_t n, int64_t nnz,
                                                     const OffT *__restrict__ off,
                                                     const int32_t *__restrict__ cols,
                                                     int32_t *counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (i < n) {
    const OffT a = off[i], b = off[i + 1];
    bad = (b < a) || (i == 0 && a != 0) || (i == n - 1 && (int64_t)b != nnz);
  }
  if (i < nnz) {
    const int32_t c = cols[i];
    bad = bad || c < 0 || c >= n;
  }
  if (bad) atomicOr(&counters[kCntRangeErr], 1);
}

__global__ void k_iota(int32_t *p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = (int32_t)i;
}

// cc[v] = v, tu[v] = tv[v] = -1
__global__ __launch_bounds__(kBlock) void k_hook_init(int64_t n, int32_t *cc, int32_t *tu,
                                                      int32_t *tv) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    cc[v] = (int32_t)v;
    tu[v] = -1;
    tv[v] = -1;
  }
}

// One block = 256 consecutive vertices; each undirected edge is hooked once,
// from its larger endpoint (arc v -> u with u < v).
template <class OffT>
__global__ __launch_bounds__(kBlock) void k_hook_light(int64_t n, const OffT *__restrict__ off,
                                                       const int32_t *__restrict__ cols,
                                                       int32_t *cc, int32_t *tu, int32_t *tv,
                                                       int64_t *chunks, int64_t chunk_cap,
                                                       int32_t *counters, int heavy_deg) {
  __shared__ int s_scan[kBlock + 1];
  __shared__ OffT s_beg[kBlock];
  __shared__ int s_wave[kBlock / kWave];
  const int t = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * kBlock;
  const int64_t v = v0 + t;
  int deg = 0;
  OffT beg = 0;
  if (v < n) {
    beg = off[v];
    const int64_t d = (int64_t)(off[v + 1] - beg);
    if (d > heavy_deg) {
      const int64_t nc = (d + kChunk - 1) / kChunk;
      const int64_t base = atomicAdd(&counters[kCntChunks], (int)nc);
      for (int64_t k = 0; k < nc && base + k < chunk_cap; ++k)
        chunks[base + k] = (v << 32) | k;
    } else {
      deg = (int)d;
    }
  }
  s_beg[t] = beg;
  int total;
  const int excl = block_excl_scan<kBlock>(deg, s_wave, &total);
  s_scan[t] = excl;
  if (t == kBlock - 1) s_scan[kBlock] = excl + deg;
  __syncthreads();
  for (int k = t; k < total; k += kBlock) {
    const int j = lds_upper_search(s_scan, kBlock, k);
    const int32_t src = (int32_t)(v0 + j);
    const int32_t dst = cols[(int64_t)s_beg[j] + (k - s_scan[j])];
    if (dst < src) hook_edge<true>(src, dst, cc, tu, tv);
  }
}

// Heavy-vertex chunks, grid-strided over the chunk list.
template <class OffT>
__global__ __launch_bounds__(kBlock) void k_hook_heavy(const OffT *__restrict__ off,
                                                       const int32_t *__restrict__ cols,
                                                       int32_t *cc, int32_t *tu, int32_t *tv,
                                                       const int64_t *chunks, int64_t chunk_cap,
                                                       const int32_t *counters) {
  int64_t nc = counters[kCntChunks];
  if (nc > chunk_cap) nc = chunk_cap;
  for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const int64_t w = chunks[c];
    const int32_t src = (int32_t)(w >> 32);
    const int64_t k = w & 0xffffffffll;
    const int64_t b = (int64_t)off[src] + k * kChunk;
    int64_t e = (int64_t)off[src + 1];
    if (e > b + kChunk) e = b + kChunk;
    for (int64_t a = b + threadIdx.x; a < e; a += kBlock) {
      const int32_t dst = cols[a];
      if (dst < src) hook_edge<true>(src, dst, cc, tu, tv);
    }
  }
}

// Edge-list hooking without recording (labels of a given forest).
__global__ __launch_bounds__(kBlock) void k_hook_coo(int64_t t, int64_t n,
                                                     const int32_t *__restrict__ eu,
                                                     const int32_t *__restrict__ ev,
                                                     int32_t *cc, int32_t *counters) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= t) return;
  const int32_t u = eu[k], v = ev[k];
  if (u < 0 || u >= n || v < 0 || v >= n) {
    atomicOr(&counters[kCntRangeErr], 1);
    return;
  }
  if (u != v) hook_edge<false>(u, v, cc, nullptr, nullptr);
}

// Final pointer jumping: every vertex points at its root (= min id of its
// component).  Also resets the per-vertex arrays the rooting stage needs.
__global__ __launch_bounds__(kBlock) void k_compress(int64_t n, int32_t *cc, int32_t *comp_root,
                                                     int32_t *head) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t r = cc[v];
  const int32_t first = r;
  int32_t nxt;
  while (r > (nxt = cc[r])) r = nxt;
  if (r != first) cc[v] = r;
  if (comp_root) comp_root[v] = -1;
  if (head) head[v] = -1;
}

// Number of components = number of vertices that are their own label.
__global__ __launch_bounds__(kBlock) void k_count_roots(int64_t n, const int32_t *__restrict__ cc,
                                                        int32_t *counters) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  wave_count(v < n && cc[v] == (int32_t)v, &counters[kCntComponents]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

rst_status enqueue_count_roots(rst_ctx *ctx, int64_t n, const int32_t *cc, int32_t *counters) {
  hipLaunchKernelGGL(k_count_roots, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, cc,
                     counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

size_t hook_chunk_capacity(const rst_ctx *ctx, int64_t nnz) {
  const int64_t heavy = ctx->opt.heavy_degree < 1 ? 1 : ctx->opt.heavy_degree;
  return (size_t)(nnz / kChunk + nnz / (heavy + 1) + 2);
}

rst_status enqueue_fill(rst_ctx *ctx, int32_t *p, int64_t count, int32_t value) {
  if (count <= 0) return RST_OK;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, kBlock)), dim3(kBlock), 0, ctx->stream,
                     p, count, value);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_validate(rst_ctx *ctx, const rst_csr *g, int32_t *counters) {
  const int64_t items = g->n > g->nnz ? g->n : g->nnz;
  if (g->offset_bytes == 4)
    hipLaunchKernelGGL(k_validate<int32_t>, dim3(grid_for(items, kBlock)), dim3(kBlock), 0,
                       ctx->stream, g->n, g->nnz, (const int32_t *)g->offsets, g->cols, counters);
  else
    hipLaunchKernelGGL(k_validate<int64_t>, dim3(grid_for(items, kBlock)), dim3(kBlock), 0,
                       ctx->stream, g->n, g->nnz, (const int64_t *)g->offsets, g->cols, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_hook_csr(rst_ctx *ctx, const rst_csr *g, ForestBufs &f, int64_t *chunks,
                            int64_t chunk_cap) {
  const int64_t n = g->n;
  hipLaunchKernelGGL(k_hook_init, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n,
                     f.cc, f.tu, f.tv);
  RST_HIP(hipGetLastError());
  const unsigned heavy_grid = (unsigned)(ctx->num_cus * 8);
  if (g->offset_bytes == 4) {
    const int32_t *off = (const int32_t *)g->offsets;
    hipLaunchKernelGGL(k_hook_light<int32_t>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0,
                       ctx->stream, n, off, g->cols, f.cc, f.tu, f.tv, chunks, chunk_cap,
                       f.counters, ctx->opt.heavy_degree);
    RST_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_hook_heavy<int32_t>, dim3(heavy_grid), dim3(kBlock), 0, ctx->stream,
                       off, g->cols, f.cc, f.tu, f.tv, chunks, chunk_cap, f.counters);
  } else {
    const int64_t *off = (const int64_t *)g->offsets;
    hipLaunchKernelGGL(k_hook_light<int64_t>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0,
                       ctx->stream, n, off, g->cols, f.cc, f.tu, f.tv, chunks, chunk_cap,
                       f.counters, ctx->opt.heavy_degree);
    RST_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_hook_heavy<int64_t>, dim3(heavy_grid), dim3(kBlock), 0, ctx->stream,
                       off, g->cols, f.cc, f.tu, f.tv, chunks, chunk_cap, f.counters);
  }
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_hook_coo(rst_ctx *ctx, int64_t n, int64_t t, const int32_t *eu,
                            const int32_t *ev, int32_t *cc, int32_t *counters) {
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, cc, n);
  RST_HIP(hipGetLastError());
  if (t > 0) {
    hipLaunchKernelGGL(k_hook_coo, dim3(grid_for(t, kBlock)), dim3(kBlock), 0, ctx->stream, t, n,
                       eu, ev, cc, counters);
    RST_HIP(hipGetLastError());
  }
  return RST_OK;
}

rst_status enqueue_compress(rst_ctx *ctx, int64_t n, int32_t *cc, int32_t *comp_root,
                            int32_t *head) {
  hipLaunchKernelGGL(k_compress, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, n, cc,
                     comp_root, head);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

}  // namespace rst
