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

// ---------------------------------------------------------------------------
// Tile phase.  One workgroup owns a tile of kTile consecutive vertex ids and
// runs union-find for the edges with both endpoints in the tile entirely in
// LDS, where compare-and-swap is cheap and coherent.  On graphs whose ids
// follow geometry (meshes, road networks) most edges are tile-internal, so
// global compare-and-swap traffic shrinks to the edges that cross tiles; those
// are appended to a list for the cross phase.  Vertices above the heavy degree
// are left to the chunked heavy pass.
//
// Inside the tile the hooking order is a fixed pseudo-random priority (a
// bijective hash of the vertex id, Sec. III-B allows any priority that avoids
// cycles): the root of lower priority is linked under the other.  Id-ordered
// hooking on a row-major mesh would build 2048-long chains that every find has
// to walk; random priorities keep trees shallow.  Afterwards every local tree
// is re-rooted at its minimum id (the edge stored at that vertex moves to the
// slot of the old root, so the set of recorded edges is unchanged) and every
// vertex points straight at that minimum: the invariant cc[x] <= x the cross
// phase relies on holds again.
// ---------------------------------------------------------------------------
constexpr int kTile = 8192;        // vertices per tile
constexpr int kTileShift = 13;
constexpr int kTileThreads = 1024;
constexpr int kTilePer = kTile / kTileThreads;

__device__ __forceinline__ uint32_t hook_priority(uint32_t x) {
  x *= 0x9E3779B1u;
  x ^= x >> 15;
  x *= 0x85EBCA77u;
  x ^= x >> 13;
  return x;   // a bijection of 32-bit values: distinct vertices never tie
}

__device__ __forceinline__ int lds_find(int x, int *lp) {
  int p = lp[x];
  while (p != x) {
    const int gp = lp[p];
    lp[x] = gp;          // path halving: x now skips to its grandparent
    x = p;
    p = gp;
  }
  return x;
}

// Cross-tile edges of tile b are written to cross[off[b*kTile] + k], a region
// as long as the tile's arc range, and counted in tile_cross[b]: no global
// atomics, no compaction.
template <class OffT>
__global__ __launch_bounds__(kTileThreads) void k_hook_tile(
    int64_t n, const OffT *__restrict__ off, const int32_t *__restrict__ cols, int32_t *cc,
    int32_t *tu, int32_t *tv, int2 *cross, int32_t *tile_cross, int32_t *counters,
    int64_t *chunks, int64_t chunk_cap, int heavy_deg) {
  __shared__ int lp[kTile];
  __shared__ int16_t eu[kTile];     // local endpoints of the edge held by a slot (-1: none)
  __shared__ int16_t ev[kTile];
  __shared__ int s_scan[kTileThreads + 1];
  __shared__ OffT s_beg[kTileThreads];
  __shared__ int s_wave[kTileThreads / kWave];
  __shared__ int s_ncross;
  const int tid = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * kTile;
  const int cnt = (int)((n - v0) < kTile ? (n - v0) : kTile);
  const int64_t region = (int64_t)off[v0];
  for (int i = tid; i < kTile; i += kTileThreads) { lp[i] = i; eu[i] = -1; ev[i] = -1; }
  if (tid == 0) s_ncross = 0;
  __syncthreads();
  for (int c = 0; c < cnt; c += kTileThreads) {
    const int li = c + tid;
    int deg = 0;
    OffT beg = 0;
    if (li < cnt) {
      const int64_t v = v0 + li;
      beg = off[v];
      const int64_t d = (int64_t)(off[v + 1] - beg);
      if (d > heavy_deg) {
        const int64_t nc = (d + kChunk - 1) / kChunk;
        const int64_t base = atomicAdd(&counters[kCntChunks], (int)nc);
        for (int64_t k = 0; k < nc && base + k < chunk_cap; ++k) chunks[base + k] = (v << 32) | k;
      } else {
        deg = (int)d;
      }
    }
    s_beg[tid] = beg;
    int total;
    const int excl = block_excl_scan<kTileThreads>(deg, s_wave, &total);
    s_scan[tid] = excl;
    if (tid == kTileThreads - 1) s_scan[kTileThreads] = excl + deg;
    __syncthreads();
    constexpr int U = 4;   // arcs in flight per thread: loads issued before any hooking
    for (int b = 0; b < total; b += kTileThreads * U) {
      int sl[U];
      int32_t dst[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = b + u * kTileThreads + tid;
        sl[u] = -1;
        dst[u] = 0;
        if (k < total) {
          const int j = lds_upper_search(s_scan, kTileThreads, k);
          sl[u] = c + j;
          dst[u] = cols[(int64_t)s_beg[j] + (k - s_scan[j])];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        bool is_cross = false;
        if (sl[u] >= 0) {
          const int64_t dl = (int64_t)dst[u] - v0;
          if (dl >= 0 && dl < sl[u]) {
            int ra = lds_find(sl[u], lp), rb = lds_find((int)dl, lp);
            while (ra != rb) {
              const bool a_low =
                  hook_priority((uint32_t)(v0 + ra)) < hook_priority((uint32_t)(v0 + rb));
              const int lo = a_low ? ra : rb, hi = a_low ? rb : ra;
              const int old = atomicCAS(&lp[lo], lo, hi);
              if (old == lo) {
                eu[lo] = (int16_t)sl[u];
                ev[lo] = (int16_t)dl;
                break;
              }
              if (ra == lo) ra = lds_find(old, lp); else rb = lds_find(old, lp);
            }
          } else {
            is_cross = dl < 0;   // dst < v0 <= src; the reverse arc is skipped
          }
        }
        const int slot = wave_append(is_cross, &s_ncross);   // LDS counter
        if (is_cross) cross[region + slot] = make_int2((int32_t)(v0 + sl[u]), dst[u]);
      }
    }
    __syncthreads();
  }
  if (tid == 0) tile_cross[blockIdx.x] = s_ncross;
  // flatten, then re-root every local tree at its minimum id.  Roots store
  // -(min+1); members lift it with atomicMax on the negated value.
  int r[kTilePer];
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int i = tid + j * kTileThreads;
    r[j] = i < cnt ? lds_find(i, lp) : i;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int i = tid + j * kTileThreads;
    if (i < cnt) lp[i] = (r[j] == i) ? -(i + 1) : r[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int i = tid + j * kTileThreads;
    if (i < cnt && r[j] != i) atomicMax(&lp[r[j]], -(i + 1));
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int i = tid + j * kTileThreads;
    if (i < cnt && r[j] == i) {
      const int m = -lp[i] - 1;
      if (m != i) {           // the old root takes the edge of the new one
        eu[i] = eu[m];
        ev[i] = ev[m];
        eu[m] = -1;
        ev[m] = -1;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int i = tid + j * kTileThreads;
    if (i < cnt) {
      const int m = -lp[r[j]] - 1;
      cc[v0 + i] = (int32_t)(v0 + m);
      const int a = eu[i];
      tu[v0 + i] = a >= 0 ? (int32_t)(v0 + a) : -1;
      tv[v0 + i] = a >= 0 ? (int32_t)(v0 + ev[i]) : -1;
    }
  }
}

// Level of a cross edge in the binary tree over tiles: tiles 2g and 2g+1 of
// level l (groups of 2^l tiles) meet at level l.  All edges inside a group
// have a smaller level, so merging level by level keeps the id-ordered trees
// of the cross phase at most one hop deeper per level.
__device__ __forceinline__ int cross_level(int32_t s, int32_t t) {
  return 31 - __clz((uint32_t)((s >> kTileShift) ^ (t >> kTileShift)));
}

// Cross phase, one level: every block walks the cross region of some tiles
// and hooks the edges of this level (asynchronous id-ordered union-find).
template <class OffT>
__global__ __launch_bounds__(kBlock) void k_hook_cross(int64_t n, const OffT *__restrict__ off,
                                                       const int2 *__restrict__ cross,
                                                       const int32_t *__restrict__ tile_cross,
                                                       int tiles, int level, int32_t *cc,
                                                       int32_t *tu, int32_t *tv) {
  for (int b = blockIdx.x; b < tiles; b += gridDim.x) {
    const int64_t region = (int64_t)off[(int64_t)b * kTile];
    const int cntb = tile_cross[b];
    for (int i = threadIdx.x; i < cntb; i += kBlock) {
      const int2 e = cross[region + i];
      if (cross_level(e.x, e.y) == level) hook_edge<true>(e.x, e.y, cc, tu, tv);
    }
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

// every arc (s -> t) with t < s may be listed, so nnz bounds the list for any CSR
size_t hook_cross_capacity(int64_t nnz) { return (size_t)(nnz + 1); }
size_t hook_tile_count(int64_t n) { return (size_t)((n + kTile - 1) / kTile); }

rst_status enqueue_hook_csr(rst_ctx *ctx, const rst_csr *g, ForestBufs &f, int64_t *chunks,
                            int64_t chunk_cap, int2 *cross, int32_t *tile_cross) {
  const int64_t n = g->n;
  const unsigned tiles = grid_for(n, kTile);
  const unsigned heavy_grid = (unsigned)(ctx->num_cus * 8);
  const unsigned cross_grid = tiles < 2048 ? tiles : 2048;
  int levels = 0;
  while ((1u << levels) < tiles) ++levels;
  if (g->offset_bytes == 4) {
    const int32_t *off = (const int32_t *)g->offsets;
    hipLaunchKernelGGL(k_hook_tile<int32_t>, dim3(tiles), dim3(kTileThreads), 0, ctx->stream, n,
                       off, g->cols, f.cc, f.tu, f.tv, cross, tile_cross, f.counters, chunks,
                       chunk_cap, ctx->opt.heavy_degree);
    RST_HIP(hipGetLastError());
    for (int l = 0; l < levels; ++l) {
      hipLaunchKernelGGL(k_hook_cross<int32_t>, dim3(cross_grid), dim3(kBlock), 0, ctx->stream, n,
                         off, cross, tile_cross, (int)tiles, l, f.cc, f.tu, f.tv);
      RST_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_hook_heavy<int32_t>, dim3(heavy_grid), dim3(kBlock), 0, ctx->stream, off,
                       g->cols, f.cc, f.tu, f.tv, chunks, chunk_cap, f.counters);
  } else {
    const int64_t *off = (const int64_t *)g->offsets;
    hipLaunchKernelGGL(k_hook_tile<int64_t>, dim3(tiles), dim3(kTileThreads), 0, ctx->stream, n,
                       off, g->cols, f.cc, f.tu, f.tv, cross, tile_cross, f.counters, chunks,
                       chunk_cap, ctx->opt.heavy_degree);
    RST_HIP(hipGetLastError());
    for (int l = 0; l < levels; ++l) {
      hipLaunchKernelGGL(k_hook_cross<int64_t>, dim3(cross_grid), dim3(kBlock), 0, ctx->stream, n,
                         off, cross, tile_cross, (int)tiles, l, f.cc, f.tu, f.tv);
      RST_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_hook_heavy<int64_t>, dim3(heavy_grid), dim3(kBlock), 0, ctx->stream, off,
                       g->cols, f.cc, f.tu, f.tv, chunks, chunk_cap, f.counters);
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
