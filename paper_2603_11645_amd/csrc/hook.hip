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

// Level of a cross edge in the binary tree over tiles: tiles 2g and 2g+1 of
// level l (groups of 2^l tiles) meet at level l.  All edges inside a group
// have a smaller level, so merging level by level keeps the id-ordered trees
// of the cross phase at most one hop deeper per level.
__device__ __forceinline__ int cross_level(int32_t s, int32_t t) {
  return 31 - __clz((uint32_t)((s >> kTileShift) ^ (t >> kTileShift)));
}

// Cross-tile edges of tile b are written to cross[off[b*kTile] + k], a region
// as long as the tile's arc range, and counted in tile_cross[b]: no global
// atomics, no compaction.
template <class OffT>
__global__ __launch_bounds__(kTileThreads) void k_hook_tile(
    int64_t n, const OffT *__restrict__ off, const int32_t *__restrict__ cols, int32_t *cc,
    int32_t *tu, int32_t *tv, int2 *cross, int32_t *tile_cross, int32_t *tile_lvl,
    int32_t *counters, int64_t *chunks, int64_t chunk_cap, int heavy_deg,
    const uint8_t *__restrict__ vmask) {
  __shared__ int lp[kTile];
  __shared__ int16_t eu[kTile];     // local endpoints of the edge held by a slot (-1: none)
  __shared__ int16_t ev[kTile];
  __shared__ int s_scan[kTile + 1]; // exclusive prefix of light degrees over the tile
  __shared__ int s_beg[kTile];      // first arc of each vertex, relative to off[v0]
  __shared__ int s_wave[kTileThreads / kWave];
  __shared__ int s_ncross, s_lmin, s_lmax;
  const int tid = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * kTile;
  const int cnt = (int)((n - v0) < kTile ? (n - v0) : kTile);
  const OffT base_off = off[v0];
  const int64_t region = (int64_t)base_off;
  for (int i = tid; i < kTile; i += kTileThreads) { lp[i] = i; eu[i] = -1; ev[i] = -1; }
  if (tid == 0) { s_ncross = 0; s_lmin = 63; s_lmax = -1; }
  // all offsets of the tile in one round trip: thread t owns vertices 8t..8t+7
  OffT o[kTilePer + 1];
#pragma unroll
  for (int j = 0; j <= kTilePer; ++j) {
    const int li = tid * kTilePer + j;
    o[j] = li <= cnt ? off[v0 + li] : (OffT)0;
  }
  int dg[kTilePer];
  int mine = 0;
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int li = tid * kTilePer + j;
    dg[j] = 0;
    // a masked vertex (its graph is handled by another method) offers no arcs
    if (li < cnt && !(vmask && vmask[v0 + li])) {
      const int64_t d = (int64_t)(o[j + 1] - o[j]);
      if (d > heavy_deg) {
        const int64_t v = v0 + li;
        const int64_t nc = (d + kChunk - 1) / kChunk;
        const int64_t cb = atomicAdd(&counters[kCntChunks], (int)nc);
        for (int64_t k = 0; k < nc && cb + k < chunk_cap; ++k) chunks[cb + k] = (v << 32) | k;
      } else {
        dg[j] = (int)d;
      }
    }
    mine += dg[j];
  }
  int total;
  int run = block_excl_scan<kTileThreads>(mine, s_wave, &total);
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int li = tid * kTilePer + j;
    s_scan[li] = run;
    s_beg[li] = (int)(o[j] - base_off);
    run += dg[j];
  }
  if (tid == 0) s_scan[kTile] = total;
  __syncthreads();
  // Arcs: thread t takes the t-th equal share of the tile's light arcs (merge
  // path over the degree scan) -- one binary search per thread, then a walk
  // along its share; loads are issued U at a time before any hooking.
  const int share = (total + kTileThreads - 1) / kTileThreads;
  const int k_begin = tid * share < total ? tid * share : total;
  const int k_end = k_begin + share < total ? k_begin + share : total;
  int j = k_begin < total ? lds_upper_search(s_scan, kTile, k_begin) : 0;
  int lvmin = 63, lvmax = -1;
  constexpr int U = 8;
  for (int kb = k_begin; kb < k_begin + share; kb += U) {
    int sl[U];
    int32_t dst[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kb + u;
      sl[u] = -1;
      dst[u] = 0;
      if (k < k_end) {
        while (s_scan[j + 1] <= k) ++j;           // next vertex with arcs left
        sl[u] = j;
        dst[u] = cols[region + s_beg[j] + (k - s_scan[j])];
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
      if (is_cross) {
        const int32_t sg = (int32_t)(v0 + sl[u]);
        cross[region + slot] = make_int2(sg, dst[u]);
        const int lv = cross_level(sg, dst[u]);
        lvmin = lv < lvmin ? lv : lvmin;
        lvmax = lv > lvmax ? lv : lvmax;
      }
    }
  }
  // level range of the tile's cross edges: reduce in the wave, one LDS atomic
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int a2 = __shfl_xor(lvmin, o, 64), b2 = __shfl_xor(lvmax, o, 64);
    lvmin = a2 < lvmin ? a2 : lvmin;
    lvmax = b2 > lvmax ? b2 : lvmax;
  }
  if ((tid & 63) == 0) {
    atomicMin(&s_lmin, lvmin);
    atomicMax(&s_lmax, lvmax);
  }
  __syncthreads();
  if (tid == 0) {
    tile_cross[blockIdx.x] = s_ncross;
    atomicAdd(&counters[kCntCross], s_ncross);
    tile_lvl[blockIdx.x] = (s_lmin << 8) | (s_lmax & 0xff);   // level range of its cross edges
  }
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

// Cross phase, one level: every block walks the cross region of some tiles
// and hooks the edges of this level (asynchronous id-ordered union-find).
// All edges along one tile boundary usually join the same two trees, so the
// block first deduplicates (root, root) pairs in an LDS hash table: only the
// first edge of a pair issues global finds-and-CAS, the rest are dropped (the
// winner's hook loop runs until the two trees are one).
constexpr int kPairSlots = 1024;
constexpr int kFlatCross = kTile;       // above this a tile's cross edges are hooked flat

__global__ __launch_bounds__(kBlock) void k_hook_cross_impl(const int64_t *__restrict__ region_of,
                                                            const int2 *__restrict__ cross,
                                                            const int32_t *__restrict__ tile_cross,
                                                            const int32_t *__restrict__ tile_lvl,
                                                            int tiles, int level, int32_t *cc,
                                                            int32_t *tu, int32_t *tv) {
  __shared__ unsigned long long tab[kPairSlots];
  for (int b = blockIdx.x; b < tiles; b += gridDim.x) {
    const int lr = tile_lvl[b];
    const int64_t region = region_of[b];
    const int cntb = tile_cross[b];
    if (cntb > kFlatCross) {
      // Many cross edges (ids without locality): pairs rarely repeat, so the
      // tile's edges are hooked directly, all levels in the first launch.
      if (level == 0)
        for (int i = threadIdx.x; i < cntb; i += kBlock) {
          const int2 e = cross[region + i];
          hook_edge<true>(e.x, e.y, cc, tu, tv);
        }
      continue;
    }
    if (level < (lr >> 8) || level > (lr & 0xff)) continue;   // block-uniform skip
    for (int i = threadIdx.x; i < kPairSlots; i += kBlock) tab[i] = ~0ull;
    __syncthreads();
    for (int i = threadIdx.x; i < cntb; i += kBlock) {
      const int2 e = cross[region + i];
      if (cross_level(e.x, e.y) != level) continue;
      const int32_t ru = find_root(e.x, cc), rv = find_root(e.y, cc);
      if (ru == rv) continue;
      const unsigned long long key = ru < rv ? ((unsigned long long)(uint32_t)ru << 32) | (uint32_t)rv
                                             : ((unsigned long long)(uint32_t)rv << 32) | (uint32_t)ru;
      uint32_t h = (uint32_t)(key * 0x9E3779B97F4A7C15ull >> 40) & (kPairSlots - 1);
      bool mine = true;
      for (int probe = 0; probe < 32; ++probe) {
        const unsigned long long old = atomicCAS(&tab[h], ~0ull, key);
        if (old == ~0ull) break;            // first edge of this pair
        if (old == key) { mine = false; break; }
        h = (h + 1) & (kPairSlots - 1);
      }
      if (mine) hook_edge<true>(e.x, e.y, cc, tu, tv);
    }
    __syncthreads();
  }
}

// region_of[b] = off[b * kTile] as int64 (so the cross kernel needs no offset type)
template <class OffT>
__global__ void k_tile_regions(const OffT *__restrict__ off, int tiles, int64_t *region_of) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < tiles) region_of[b] = (int64_t)off[(int64_t)b * kTile];
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
int hook_level_count(int64_t n) {
  int l = 0;
  while (((size_t)1 << l) < hook_tile_count(n)) ++l;
  return l;
}
// tile_cross buffer: int32 counts, int64 region starts, int32 level ranges
size_t hook_tile_words(int64_t n) { return ((hook_tile_count(n) + 1) & ~size_t(1)) + 3 * hook_tile_count(n); }

static rst_status launch_cross_levels(rst_ctx *ctx, unsigned tiles, int levels, unsigned grid,
                                      const int64_t *region_of, const int2 *cross,
                                      const int32_t *tile_cross, const int32_t *tile_lvl,
                                      ForestBufs &f) {
  RST_KMARK(ctx, RST_KERNEL_CROSS, 0);
  for (int l = 0; l < levels; ++l) {
    hipLaunchKernelGGL(k_hook_cross_impl, dim3(grid), dim3(kBlock), 0, ctx->stream, region_of, cross,
                       tile_cross, tile_lvl, (int)tiles, l, f.cc, f.tu, f.tv);
    RST_HIP(hipGetLastError());
  }
  RST_KMARK(ctx, RST_KERNEL_CROSS, 1);
  return RST_OK;
}

rst_status enqueue_hook_csr(rst_ctx *ctx, const rst_csr *g, ForestBufs &f, int64_t *chunks,
                            int64_t chunk_cap, int2 *cross, int32_t *tile_cross) {
  const size_t tc = hook_tile_count(g->n);
  int64_t *region_of = reinterpret_cast<int64_t *>(tile_cross + ((tc + 1) & ~size_t(1)));
  int32_t *tile_lvl = reinterpret_cast<int32_t *>(region_of + tc);
  const int64_t n = g->n;
  const unsigned tiles = grid_for(n, kTile);
  const unsigned heavy_grid = (unsigned)(ctx->num_cus * 8);
  const unsigned cross_grid = tiles < 2048 ? tiles : 2048;
  int levels = 0;
  while ((1u << levels) < tiles) ++levels;
  if (g->offset_bytes == 4) {
    const int32_t *off = (const int32_t *)g->offsets;
    RST_KMARK(ctx, RST_KERNEL_HOOK_TILE, 0);
    hipLaunchKernelGGL(k_hook_tile<int32_t>, dim3(tiles), dim3(kTileThreads), 0, ctx->stream, n,
                       off, g->cols, f.cc, f.tu, f.tv, cross, tile_cross, tile_lvl, f.counters,
                       chunks, chunk_cap, ctx->opt.heavy_degree, f.vmask);
    RST_HIP(hipGetLastError());
    RST_KMARK(ctx, RST_KERNEL_HOOK_TILE, 1);
    hipLaunchKernelGGL(k_tile_regions<int32_t>, dim3(grid_for(tiles, kBlock)), dim3(kBlock), 0,
                       ctx->stream, off, (int)tiles, region_of);
    RST_HIP(hipGetLastError());
    RST_TRY(launch_cross_levels(ctx, tiles, levels, cross_grid, region_of, cross, tile_cross,
                                tile_lvl, f));
    hipLaunchKernelGGL(k_hook_heavy<int32_t>, dim3(heavy_grid), dim3(kBlock), 0, ctx->stream, off,
                       g->cols, f.cc, f.tu, f.tv, chunks, chunk_cap, f.counters);
  } else {
    const int64_t *off = (const int64_t *)g->offsets;
    RST_KMARK(ctx, RST_KERNEL_HOOK_TILE, 0);
    hipLaunchKernelGGL(k_hook_tile<int64_t>, dim3(tiles), dim3(kTileThreads), 0, ctx->stream, n,
                       off, g->cols, f.cc, f.tu, f.tv, cross, tile_cross, tile_lvl, f.counters,
                       chunks, chunk_cap, ctx->opt.heavy_degree, f.vmask);
    RST_HIP(hipGetLastError());
    RST_KMARK(ctx, RST_KERNEL_HOOK_TILE, 1);
    hipLaunchKernelGGL(k_tile_regions<int64_t>, dim3(grid_for(tiles, kBlock)), dim3(kBlock), 0,
                       ctx->stream, off, (int)tiles, region_of);
    RST_HIP(hipGetLastError());
    RST_TRY(launch_cross_levels(ctx, tiles, levels, cross_grid, region_of, cross, tile_cross,
                                tile_lvl, f));
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
