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
#include "unionfind.h"

namespace rst {

constexpr int kChunk = 4096;   // arcs per heavy-vertex chunk

// ---------------------------------------------------------------------------
// kernels (the union-find steps themselves are in unionfind.h)
// ---------------------------------------------------------------------------

// counters[0..31] = 0 and counters[32] = root (the one-root buffer) in one launch
__global__ void k_reset_counters(int32_t *counters, int32_t root) {
  const int i = threadIdx.x;
  if (i < 32) counters[i] = 0;
  else if (i == 32) counters[32] = root;
}

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
  if (i < count) store_agent(&p[i], (int32_t)i);
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
// Inside the tile the hooking order is a fixed priority that scatters
// neighbouring ids (the bit reversal of the tile-local id, a bijection; Sec.
// III-B allows any priority that avoids cycles): the root of lower priority is
// linked under the other.  Id-ordered hooking on a row-major mesh would build
// 2048-long chains that every find has to walk; a scattering priority keeps
// trees shallow.  (The kernel is bound by its vector instructions: the bit
// reversal, one instruction, replaced a multiplicative hash and cut it 4%.)  Afterwards every local tree
// is re-rooted at its minimum id (the edge stored at that vertex moves to the
// slot of the old root, so the set of recorded edges is unchanged) and every
// vertex points straight at that minimum: the invariant cc[x] <= x the cross
// phase relies on holds again.
// ---------------------------------------------------------------------------
constexpr int kTile = 8192;        // vertices per tile
constexpr int kTileShift = 13;
constexpr int kTileThreads = 1024;
constexpr int kTilePer = kTile / kTileThreads;

// vertices per group of the tile's degree prefix, and the largest degree a
// vertex may have to be hooked by its tile (its arcs beyond would not fit the
// 16-bit in-group prefix; such a vertex goes to the chunked heavy pass)
constexpr int kTileGroup = 64;
constexpr int kTileLightMax = 1023;
constexpr int kTileMask = kTile - 1;

// LDS word of a tile vertex while hooking: its parent in the low 13 bits and,
// once it has been hooked as a root, 1 + the local source of the hooking edge
// above them (the edge's other end is kept in ev[]).  Path halving rewrites
// the parent bits only; a non-root's upper bits never change again.
__device__ __forceinline__ int lds_find_tile(int x, int *lp) {
  int w = lp[x];
  int p = w & kTileMask;
  while (p != x) {
    const int wp = lp[p];
    const int gp = wp & kTileMask;
    lp[x] = (w & ~kTileMask) | gp;   // path halving: x now skips to its grandparent
    x = p;
    w = wp;
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
//
// LDS (64.6 KB, two workgroups per CU): lp, the hooking words, later the tree
// minima, then the heads of the tile's arc lists; s16, first the in-group
// degree prefix and ev (other end of each root's hooking edge), then eu and ev,
// then the tile's next-arc links; the group bases of the degree prefix.
template <class OffT>
__global__ __launch_bounds__(kTileThreads, 8) void k_hook_tile(
    int64_t n, const OffT *__restrict__ off, const int32_t *__restrict__ cols, int32_t *cc,
    int32_t *tu, int32_t *tv, int2 *cross, int32_t *tile_cross, int32_t *tile_lvl,
    int64_t *region_of, int32_t *counters, int64_t *chunks, int64_t chunk_cap, int heavy_deg,
    const uint8_t *__restrict__ vmask, int32_t *head, int32_t *next, int vec_cols,
    const uint8_t *__restrict__ gsel) {
  __shared__ int lp[kTile];
  __shared__ __align__(16) int16_t s16[2 * kTile];
  __shared__ int s_gbase[kTile / kTileGroup + 1];   // light arcs before each group; [last] = all
  __shared__ int s_wave[kTileThreads / kWave];
  __shared__ int s_ncross, s_lmin, s_lmax, s_gap;
  uint16_t *sc16 = reinterpret_cast<uint16_t *>(s16);   // light arcs before a vertex, in its group
  int16_t *eu = s16;                                     // after the arcs: source of each root's edge
  int16_t *ev = s16 + kTile;
  const int tid = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * kTile;
  const int cnt = (int)((n - v0) < kTile ? (n - v0) : kTile);
  const OffT base_off = off[v0];
  const int64_t region = (int64_t)base_off;
  const int light_max = heavy_deg < kTileLightMax ? heavy_deg : kTileLightMax;
  for (int i = tid; i < kTile; i += kTileThreads) { lp[i] = i; ev[i] = -1; }
  if (tid == 0) { s_ncross = 0; s_lmin = 63; s_lmax = -1; s_gap = 0; }
  // all offsets of the tile in one round trip: thread t owns vertices 8t..8t+7
  // (read as 16-byte vectors when the offsets are 16-byte aligned)
  OffT o[kTilePer + 1];
  if ((vec_cols & 2) && tid * kTilePer + kTilePer <= cnt) {
    const int4 *o4 = reinterpret_cast<const int4 *>(off + v0 + tid * kTilePer);
    constexpr int PV = 16 / (int)sizeof(OffT);
#pragma unroll
    for (int q = 0; q < kTilePer / PV; ++q) {
      const int4 w = o4[q];
      if (PV == 4) {
        o[4 * q] = (OffT)w.x; o[4 * q + 1] = (OffT)w.y;
        o[4 * q + 2] = (OffT)w.z; o[4 * q + 3] = (OffT)w.w;
      } else {
        o[2 * q] = (OffT)(((uint64_t)(uint32_t)w.y << 32) | (uint32_t)w.x);
        o[2 * q + 1] = (OffT)(((uint64_t)(uint32_t)w.w << 32) | (uint32_t)w.z);
      }
    }
    o[kTilePer] = off[v0 + tid * kTilePer + kTilePer];
  } else {
#pragma unroll
    for (int j = 0; j <= kTilePer; ++j) {
      const int li = tid * kTilePer + j;
      o[j] = li <= cnt ? off[v0 + li] : (OffT)0;
    }
  }
  int dg[kTilePer];
  int mine = 0;
  bool gap = false;
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int li = tid * kTilePer + j;
    dg[j] = 0;
    // a masked vertex (its graph is handled by another method, or hooked by
    // the global sweep) offers no arcs
    if (li < cnt && !(vmask && vmask[v0 + li]) && !(gsel && gsel[v0 + li])) {
      const int64_t d = (int64_t)(o[j + 1] - o[j]);
      if (d > light_max) {
        const int64_t v = v0 + li;
        const int64_t nc = (d + kChunk - 1) / kChunk;
        const int64_t cb = atomicAdd(&counters[kCntChunks], (int)nc);
        for (int64_t k = 0; k < nc && cb + k < chunk_cap; ++k) chunks[cb + k] = (v << 32) | k;
      } else {
        dg[j] = (int)d;
      }
    }
    // s_gap: some vertex offers fewer arcs than it has (heavy or masked), so
    // the light arcs are not one contiguous range of cols
    gap |= li < cnt && (int64_t)dg[j] != (int64_t)(o[j + 1] - o[j]);
    mine += dg[j];
  }
  int total;
  const int run0 = block_excl_scan<kTileThreads>(mine, s_wave, &total);
  // the 8 threads of a 64-vertex group sit in one wave: the group's base is
  // the prefix of its first thread
  const int gb = __shfl(run0, (tid & 63) & ~(kTileGroup / kTilePer - 1), 64);
  if ((tid & (kTileGroup / kTilePer - 1)) == 0) s_gbase[tid / (kTileGroup / kTilePer)] = run0;
  if (tid == 0) s_gbase[kTile / kTileGroup] = total;
  int run = run0 - gb;
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    sc16[tid * kTilePer + j] = (uint16_t)run;
    run += dg[j];
  }
  if (gap) s_gap = 1;
  __syncthreads();
  // light arcs before vertex j of the tile (j = kTile: all of them)
  auto scan_at = [&](int q) -> int {
    return s_gbase[q / kTileGroup] + (q < kTile ? (int)sc16[q] : 0);
  };
  // Arcs: thread t takes the t-th equal share of the tile's light arcs (merge
  // path over the degree prefix) -- one binary search per thread, then a walk
  // along its share.
  const int share = (total + kTileThreads - 1) / kTileThreads;
  const int k_begin = tid * share < total ? tid * share : total;
  const int k_end = k_begin + share < total ? k_begin + share : total;
  int j = 0;
  if (k_begin < total) {
    int lo = 0, hi = kTile;   // largest j with scan_at(j) <= k_begin
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (scan_at(mid) <= k_begin) lo = mid; else hi = mid;
    }
    j = lo;
  }
  int next_start = scan_at(j + 1);
  int lvmin = 63, lvmax = -1;
  // Arc (v0 + src) -> dst: hook it if both ends lie in the tile (one of the
  // two arcs of an edge does it); true if it is a cross arc to keep, i.e.
  // dst < v0 <= src (the reverse arc is skipped).
  const int32_t v0i = (int32_t)v0;   // ids are below 2^31
  auto visit = [&](int src, int32_t dst) -> bool {
    const int32_t dl = dst - v0i;
    if ((uint32_t)dl < (uint32_t)src) {
      // same parent, or one the other's parent: same tree, no walk needed
      const int pa = lp[src] & kTileMask, pb = lp[dl] & kTileMask;
      if (pa == pb || pa == (int)dl || pb == src) return false;
      int ra = lds_find_tile(pa, lp), rb = lds_find_tile(pb, lp);
      while (ra != rb) {
        // priority: bit reversal of the local id (distinct ids never tie)
        const bool a_low = __builtin_bitreverse32((uint32_t)ra) < __builtin_bitreverse32((uint32_t)rb);
        const int lo = a_low ? ra : rb, hi = a_low ? rb : ra;
        const int old = atomicCAS(&lp[lo], lo, hi | ((src + 1) << kTileShift));
        if (old == lo) {
          ev[lo] = (int16_t)dl;
          break;
        }
        const int np = lds_find_tile(old & kTileMask, lp);
        if (ra == lo) ra = np; else rb = np;
      }
      return false;
    }
    return dl < 0;
  };
  auto keep_cross = [&](int slot, int src, int32_t dst) {
    const int32_t sg = (int32_t)(v0 + src);
    cross[region + slot] = make_int2(sg, dst);
    const int lv = cross_level(sg, dst);
    lvmin = lv < lvmin ? lv : lvmin;
    lvmax = lv > lvmax ? lv : lvmax;
  };
  if (!s_gap) {
    // The share is the contiguous range [region + k_begin, region + k_end) of
    // cols: read 16 arcs at a time, as aligned 16-byte vectors when cols is
    // 16-byte aligned (the vectors may reach into the neighbours' shares,
    // never past the tile's arcs).  Cross arcs are appended four arcs at a
    // time, one LDS atomic per wave for all four.
    const int64_t p0 = region + k_begin, p1 = region + k_end, pend = region + total;
    constexpr int V = 4;
    // the same trip count in every lane (the ballots below need the whole wave)
    const int nit = (share + 3 + 4 * V - 1) / (4 * V);
    // tile-local arc index of the first vector (the share's start rounded down
    // to 4 arcs; in-range tests below in 32 bits)
    const int ka = (int)((p0 & ~(int64_t)3) - region);
    for (int it = 0; it < nit; ++it) {
      const int64_t pa = (p0 & ~(int64_t)3) + (int64_t)it * (4 * V);
      int32_t cv[4 * V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int64_t q = pa + 4 * v;
        if ((vec_cols & 1) && q + 4 <= pend) {
          const int4 x = *reinterpret_cast<const int4 *>(cols + q);
          cv[4 * v] = x.x; cv[4 * v + 1] = x.y; cv[4 * v + 2] = x.z; cv[4 * v + 3] = x.w;
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) cv[4 * v + c] = (q + c >= p0 && q + c < p1) ? cols[q + c] : 0;
        }
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        bool isc[4];
        int js[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int k = ka + it * (4 * V) + 4 * v + c;
          isc[c] = false;
          js[c] = 0;
          if (k >= k_begin && k < k_end) {
            while (next_start <= k) next_start = scan_at(++j + 1);   // next vertex with arcs left
            js[c] = j;
            isc[c] = visit(j, cv[4 * v + c]);
          }
        }
        uint64_t m[4];
        int tot = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) { m[c] = __ballot(isc[c]); tot += (int)__popcll(m[c]); }
        if (tot) {
          int base = 0;
          if ((tid & 63) == 0) base = atomicAdd(&s_ncross, tot);
          base = __shfl(base, 0, 64);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (isc[c]) keep_cross(base + lanes_below(m[c]), js[c], cv[4 * v + c]);
            base += (int)__popcll(m[c]);
          }
        }
      }
    }
  } else {
    // heavy or masked vertices: arc k of vertex j is cols[off[v0 + j] + k -
    // scan_at(j)].  The thread keeps the offset of its current vertex and has
    // the next one's in flight, so a batch of U arcs costs one round trip
    // unless the walk passes several vertices in it.
    constexpr int U = 4;
    int cur_start = scan_at(j);
    int64_t ob_cur = (int64_t)off[v0 + j];
    int64_t ob_next = (int64_t)off[v0 + j + 1];   // j < cnt, so v0 + j + 1 <= n
    for (int kb = k_begin; kb < k_begin + share; kb += U) {
      int sl[U];
      int64_t ci[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = kb + u;
        sl[u] = -1;
        ci[u] = 0;
        if (k < k_end) {
          if (next_start <= k) {
            int jn = j;
            while (next_start <= k) { cur_start = next_start; next_start = scan_at(++jn + 1); }
            ob_cur = jn == j + 1 ? ob_next : (int64_t)off[v0 + jn];
            j = jn;
            ob_next = (int64_t)off[v0 + j + 1];
          }
          sl[u] = j;
          ci[u] = ob_cur + (k - cur_start);
        }
      }
      int32_t dst[U];
#pragma unroll
      for (int u = 0; u < U; ++u) dst[u] = sl[u] >= 0 ? cols[ci[u]] : 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool is_cross = sl[u] >= 0 && visit(sl[u], dst[u]);
        const int slot = wave_append(is_cross, &s_ncross);   // LDS counter
        if (is_cross) keep_cross(slot, sl[u], dst[u]);
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
    if (blockIdx.x == 0) {   // read by the cross phase after this kernel
      counters[kCntKept] = 0;
      counters[kCntKeptTop] = 0;
      counters[kCntCrossDone] = 0;
      counters[kCntCrossOverflow] = 0;
    }
    region_of[blockIdx.x] = region;
    tile_cross[blockIdx.x] = s_ncross;
    atomicAdd(&counters[kCntCross], s_ncross);
    tile_lvl[blockIdx.x] = (s_lmin << 8) | (s_lmax & 0xff);   // level range of its cross edges
  }
  // flatten, then re-root every local tree at its minimum id.  Roots store
  // -(min+1); members lift it with atomicMax on the negated value.
  int r[kTilePer];
#pragma unroll
  for (int j2 = 0; j2 < kTilePer; ++j2) {
    const int i = tid + j2 * kTileThreads;
    r[j2] = i < cnt ? lds_find_tile(i, lp) : i;
  }
  __syncthreads();
  // the degree prefix is done with: the sources of the hooking edges move out
  // of the words into eu
#pragma unroll
  for (int j2 = 0; j2 < kTilePer; ++j2) {
    const int i = tid + j2 * kTileThreads;
    if (i < cnt) {
      eu[i] = (int16_t)((lp[i] >> kTileShift) - 1);
      lp[i] = (r[j2] == i) ? -(i + 1) : r[j2];
    }
  }
  __syncthreads();
  // Only the first lane of a run of lanes with the same root does the atomic
  // (it holds the run's smallest id): on a mesh tile nearly every vertex has
  // the same root, and 8192 atomics on one LDS word serialise.
#pragma unroll
  for (int j2 = 0; j2 < kTilePer; ++j2) {
    const int i = tid + j2 * kTileThreads;
    const int left = __shfl_up(r[j2], 1, 64);
    const bool first = (tid & 63) == 0 || left != r[j2];
    if (i < cnt && r[j2] != i && first) atomicMax(&lp[r[j2]], -(i + 1));
  }
  __syncthreads();
#pragma unroll
  for (int j2 = 0; j2 < kTilePer; ++j2) {
    const int i = tid + j2 * kTileThreads;
    if (i < cnt && r[j2] == i) {
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
  int ea[kTilePer], eb[kTilePer];
#pragma unroll
  for (int j2 = 0; j2 < kTilePer; ++j2) {
    const int i = tid + j2 * kTileThreads;
    ea[j2] = -1;
    eb[j2] = -1;
    if (i < cnt) {
      const int m = -lp[r[j2]] - 1;
      store_agent(&cc[v0 + i], (int32_t)(v0 + m));
      ea[j2] = eu[i];
      eb[j2] = ev[i];
      tu[v0 + i] = ea[j2] >= 0 ? (int32_t)(v0 + ea[j2]) : -1;
      tv[v0 + i] = ea[j2] >= 0 ? (int32_t)(v0 + eb[j2]) : -1;
    }
  }
  if (!head) return;
  // Euler arc lists of the tile's own edges, built in LDS and written once,
  // coalesced: local arc 2i / 2i+1 of slot i is global arc 2(v0+i) / 2(v0+i)+1.
  __syncthreads();                                      // lp, eu, ev read by all
  int *lhead = lp;                                      // [kTile] first local arc
  int16_t *lnext = s16;                                 // [2 kTile] next local arc
  for (int i = tid; i < kTile; i += kTileThreads) lhead[i] = -1;
  __syncthreads();
#pragma unroll
  for (int j2 = 0; j2 < kTilePer; ++j2) {
    const int i = tid + j2 * kTileThreads;
    if (i < cnt) {
      int16_t n0 = -1, n1 = -1;
      if (ea[j2] >= 0) {
        n0 = (int16_t)atomicExch(&lhead[ea[j2]], 2 * i);
        n1 = (int16_t)atomicExch(&lhead[eb[j2]], 2 * i + 1);
      }
      lnext[2 * i] = n0;
      lnext[2 * i + 1] = n1;
    }
  }
  __syncthreads();
  const int32_t arc0 = (int32_t)(2 * v0);
#pragma unroll
  for (int j2 = 0; j2 < kTilePer; ++j2) {
    const int i = tid + j2 * kTileThreads;
    if (i < cnt) {
      const int h = lhead[i];
      store_agent(&head[v0 + i], h >= 0 ? arc0 + h : -1);
      const int n0 = lnext[2 * i], n1 = lnext[2 * i + 1];
      reinterpret_cast<int2 *>(next)[v0 + i] =
          make_int2(n0 >= 0 ? arc0 + n0 : -1, n1 >= 0 ? arc0 + n1 : -1);
    }
  }
}

// Cross phase.  After the tile pass every vertex points at its tile-local
// root, and the cross edges of a tile mostly join the same few pairs of local
// trees (on a mesh, one big tree per tile and some small ones along its
// borders).  The phase runs in steps:
//  1. k_cross_dedupe: every cross edge (s,t) of a tile is keyed by the pair of
//     trees it joins, (cc[s], cc[t]), and only the first edge of each pair is
//     kept, compacted in place at the start of the tile's region;
//     tile_cross[b] becomes the number kept.  A tile with more than
//     kFlatCross cross edges has no locality to exploit: its edges are hooked
//     right there (split over several blocks) and tile_cross[b] keeps its
//     original value, which marks the tile as done for the later steps.
//  2. k_cross_lds: the levels of the binary tree of tiles (cross_level) below
//     `split` are merged by one block per group of 2^split tiles, the rest by
//     one block from a list of their edges: a block maps the roots its kept
//     edges join into LDS, runs the union-find there and writes the links
//     back.  With few kept edges, one block takes all levels.  A block whose
//     edges or roots do not fit changes nothing and raises a flag.
//  3. Only when flagged, k_late_hooks hooks every kept edge in global memory
//     by compare-and-swap, spread over the whole grid.
// Splitting by levels keeps each group's roots inside its own tiles, so the
// group merges are independent.  A key read while another tile hooks may already be an
// ancestor of the local root rather than the root itself: both name a vertex
// of the same current tree, so dropping an edge with an equal key never loses
// connectivity.
constexpr int kDedupSlots = 8192;       // LDS hash slots (64 KB) of k_cross_dedupe
constexpr int kFlatCross = kTile;       // above this a tile's cross edges are hooked flat
constexpr int kDedupPer = kFlatCross / kTileThreads;
constexpr int kLdsSlots = 8192;         // root slots of k_cross_lds (key + parent: 64 KB)
constexpr int kLdsPer = 16;             // kept edges per thread in k_cross_lds
constexpr int kLdsEdges = kLdsPer * kTileThreads;
// The one-block merge of all levels takes at most this many kept edges: one
// CU gathers about a cache line per clock, so longer lists go faster through
// the group merges spread over many CUs.
constexpr int kAllEdges = 2048;

__device__ __forceinline__ int kept_count(int c) { return c > kFlatCross ? 0 : c; }

__global__ __launch_bounds__(kTileThreads, 8) void k_cross_dedupe(const int64_t *__restrict__ region_of,
                                                               int2 *cross, int32_t *tile_cross,
                                                               int slices, int32_t *cc, int32_t *tu,
                                                               int32_t *tv, int32_t *counters,
                                                               int2 *kept_list, int split,
                                                               int32_t *head, int32_t *next) {
  __shared__ unsigned long long tab[kDedupSlots];
  __shared__ int s_kept, s_top, s_base, s_base_all;
  const int b = blockIdx.x / slices;
  const int part = blockIdx.x % slices;
  const int tid = threadIdx.x;
  const int64_t region = region_of[b];
  const int cntb = tile_cross[b];
  if (cntb > kFlatCross) {
    for (int i = part * kTileThreads + tid; i < cntb; i += slices * kTileThreads) {
      const int2 e = cross[region + i];
      hook_edge<true>(e.x, e.y, cc, tu, tv, head, next);
    }
    block_release_device();
    return;
  }
  if (part != 0) return;
  for (int i = tid; i < kDedupSlots; i += kTileThreads) tab[i] = ~0ull;
  if (tid == 0) { s_kept = 0; s_top = 0; }
  // every edge of the tile is read (and its key formed) before any write-back
  int2 e[kDedupPer];
  bool keep[kDedupPer];
#pragma unroll
  for (int j = 0; j < kDedupPer; ++j) {
    const int i = tid + j * kTileThreads;
    e[j] = i < cntb ? cross[region + i] : make_int2(0, 0);
  }
  int32_t ka[kDedupPer], kb[kDedupPer];
#pragma unroll
  for (int j = 0; j < kDedupPer; ++j) {
    const int i = tid + j * kTileThreads;
    ka[j] = i < cntb ? cc[e[j].x] : 0;
    kb[j] = i < cntb ? cc[e[j].y] : 0;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kDedupPer; ++j) {
    const int i = tid + j * kTileThreads;
    keep[j] = false;
    if (i < cntb && ka[j] != kb[j]) {
      const uint32_t lo = (uint32_t)(ka[j] < kb[j] ? ka[j] : kb[j]);
      const uint32_t hi = (uint32_t)(ka[j] < kb[j] ? kb[j] : ka[j]);
      const unsigned long long key = ((unsigned long long)lo << 32) | hi;
      uint32_t h = (uint32_t)(key * 0x9E3779B97F4A7C15ull >> 40) & (kDedupSlots - 1);
      keep[j] = true;                   // also kept when the probe limit is hit
      for (int probe = 0; probe < 64; ++probe) {
        const unsigned long long old = atomicCAS(&tab[h], ~0ull, key);
        if (old == ~0ull) break;        // first edge of this pair
        if (old == key) { keep[j] = false; break; }
        h = (h + 1) & (kDedupSlots - 1);
      }
    }
  }
  __syncthreads();
  int slot[kDedupPer], slot_all[kDedupPer];
#pragma unroll
  for (int j = 0; j < kDedupPer; ++j) {
    const int k = wave_append(keep[j], &s_kept);
    if (keep[j]) cross[region + k] = e[j];
    slot_all[j] = keep[j] ? k : -1;
    const bool top = keep[j] && cross_level(e[j].x, e[j].y) >= split;
    slot[j] = wave_append(top, &s_top);
    if (!top) slot[j] = -1;
  }
  __syncthreads();
  // Every kept edge also goes to one compact list (tiles in any order) for the
  // one-workgroup merge of all levels, and those of the levels >= split to a
  // second one for the top-level merge; a list past kLdsEdges is not used.
  if (tid == 0) {
    tile_cross[b] = s_kept;
    // both list bases from one 8-byte atomic (512 blocks queue on one word)
    static_assert(kCntKeptTop == kCntKept + 1 && kCntKept % 2 == 0, "kept counters share a word");
    const unsigned long long old =
        s_kept ? atomicAdd(reinterpret_cast<unsigned long long *>(&counters[kCntKept]),
                           ((unsigned long long)(uint32_t)s_top << 32) | (uint32_t)s_kept)
               : 0ull;
    s_base_all = (int)(uint32_t)old;
    s_base = (int)(uint32_t)(old >> 32);
  }
  __syncthreads();
  const int kba = s_base_all;
  if (kba + s_kept <= kLdsEdges) {
#pragma unroll
    for (int j = 0; j < kDedupPer; ++j)
      if (slot_all[j] >= 0) kept_list[kba + slot_all[j]] = e[j];
  }
  const int kb0 = s_base;
  int2 *kept_top = kept_list + kLdsEdges;
  if (kb0 + s_top <= kLdsEdges) {
#pragma unroll
    for (int j = 0; j < kDedupPer; ++j)
      if (slot[j] >= 0) kept_top[kb0 + slot[j]] = e[j];
  }
}

// Slot of global root `key` in the LDS table (inserted if new); -1 when the
// probe limit is reached.
__device__ __forceinline__ int lds_slot(int32_t key, int32_t *keys) {
  uint32_t h = ((uint32_t)key * 0x9E3779B1u) >> (32 - 13);
  for (int probe = 0; probe < 256; ++probe) {
    const int32_t old = atomicCAS(&keys[h], -1, key);
    if (old == -1 || old == key) return (int)h;
    h = (h + 1) & (kLdsSlots - 1);
  }
  return -1;
}
static_assert(kLdsSlots == 1 << 13, "lds_slot hashes to 13 bits");

// LDS union-find entries of k_cross_lds: parent slot in the low 14 bits; a
// hooked slot also keeps 1 + the number of the kept edge that hooked it in
// the bits above (roots hold just their own slot).  Path halving rewrites the
// parent bits only.
constexpr int kParMask = 0x3fff;

__device__ __forceinline__ int lds_find_rec(int x, int *par) {
  int w = par[x];
  int p = w & kParMask;
  while (p != x) {
    const int wp = par[p];
    const int gp = wp & kParMask;
    par[x] = (w & ~kParMask) | gp;   // x's hook record is immutable, kept as is
    x = p;
    w = wp;
    p = gp;
  }
  return x;
}

// One union in the LDS table (smaller global id wins); the winner of the
// compare-and-swap stores the kept edge number g with the new parent and adds
// the hooked slot to the list `hooks`.
__device__ __forceinline__ void lds_union(int sa, int sb, int g, const int32_t *keys, int *par,
                                          int *hooks, int *nhooks) {
  int ra = lds_find_rec(sa, par), rb = lds_find_rec(sb, par);
  while (ra != rb) {
    const bool a_low = keys[ra] < keys[rb];
    const int lo = a_low ? ra : rb, hi = a_low ? rb : ra;
    const int old = atomicCAS(&par[hi], hi, lo | ((g + 1) << 14));
    if (old == hi) {
      hooks[atomicAdd(nhooks, 1)] = hi;   // each slot is hooked once
      return;
    }
    const int np = lds_find_rec(old & kParMask, par);
    if (ra == hi) ra = np; else rb = np;
  }
}

// Packed per-edge state of k_cross_lds: root slots (14 bits each) and level
// (4 bits, below 15); ~0u marks no edge.
__device__ __forceinline__ uint32_t pack_sab(int sa, int sb, int level) {
  return (uint32_t)sa | ((uint32_t)sb << 14) | ((uint32_t)level << 28);
}

// One-workgroup LDS merge of the kept cross edges of levels [lo, hi).
// kGroup: block g takes the tiles [g << group_log, (g + 1) << group_log) and
// their kept edges below hi (their roots must lie in the group's vertex range,
// else the block raises the flag and changes nothing) -- unless there are at
// most kAllEdges kept edges: then block 0 alone takes all of them, levels
// [0, all_hi), sets counters[kCntCrossDone] so that the top-level merge
// returns at once, and raises the flag if they do not fit.  Otherwise (one
// block) the compact list of the edges of the top levels.
template <bool kGroup>
__global__ __launch_bounds__(kTileThreads) void k_cross_lds(const int64_t *__restrict__ region_of,
                                                            const int2 *__restrict__ cross,
                                                            const int32_t *__restrict__ tile_cross,
                                                            const int2 *__restrict__ kept_list,
                                                            int tiles, int lo, int hi,
                                                            int group_log, int all_hi,
                                                            int32_t *cc, int32_t *tu, int32_t *tv,
                                                            int32_t *counters, int32_t *head,
                                                            int32_t *next) {
  __shared__ int32_t keys[kLdsSlots];   // global root held by a slot, -1: empty
  __shared__ int par[kLdsSlots];        // union-find entries (see kParMask)
  __shared__ int s_hooks[kLdsSlots];    // slots hooked by the unions
  __shared__ int s_pref[kGroup ? kTileThreads + 1 : 1];   // kept counts of the group's tiles
  __shared__ int s_wave[kTileThreads / kWave];
  __shared__ int s_fail, s_nhooks;
  const int tid = threadIdx.x;
  // every branch below is block-uniform
  const bool all = kGroup && counters[kCntKept] <= kAllEdges;
  if (all && blockIdx.x != 0) return;
  if (!kGroup && counters[kCntCrossDone]) return;
  const bool grp = kGroup && !all;
  if (all) { lo = 0; hi = all_hi; }
  const int64_t t0 = grp ? ((int64_t)blockIdx.x << group_log) : 0;
  const int64_t t1 = grp ? ((t0 + ((int64_t)1 << group_log)) < tiles
                                ? t0 + ((int64_t)1 << group_log) : (int64_t)tiles) : 0;
  int total;
  // a group block takes its edges from the list of all kept edges when that
  // list is complete (it then filters by level and group), else from its
  // tiles' regions of the cross list
  const bool from_list = !grp || counters[kCntKept] <= kLdsEdges;
  const int2 *list = kept_list + (kGroup ? 0 : kLdsEdges);
  if (all || (grp && from_list)) {
    total = counters[kCntKept];
  } else if (grp) {
    const int64_t tb = t0 + tid;
    const int c = tb < t1 ? kept_count(tile_cross[tb]) : 0;
    const int ex = block_excl_scan<kTileThreads>(c, s_wave, &total);
    s_pref[tid] = ex;
  } else {
    total = counters[kCntKeptTop];
  }
  if (total > kLdsEdges) {
    if (tid == 0) counters[kCntCrossOverflow] = 1;
    return;
  }
  if (total == 0) return;
  for (int i = tid; i < kLdsSlots; i += kTileThreads) { keys[i] = -1; par[i] = i; }
  if (tid == 0) { s_fail = 0; s_nhooks = 0; }
  __syncthreads();
  const int32_t own_lo = grp ? (int32_t)(t0 << kTileShift) : 0;
  const int32_t own_hi = grp ? (int32_t)((t1 << kTileShift) - 1) : 0x7fffffff;
  auto edge_at = [&](int g) -> int2 {
    if (from_list) return list[g];
    const int k = lds_upper_search(s_pref, kTileThreads, g);
    return cross[region_of[t0 + k] + (g - s_pref[k])];
  };
  // Edge g = tid + k * kTileThreads is this thread's k-th.  The roots it joins
  // are found with the first two hops of a batch of edges issued together
  // (one hop reaches the tile-local root, usually a root already); only the
  // rest walk on.  No other block writes these roots now, so the finds end at
  // true roots.
  uint32_t sab[kLdsPer];                // pack_sab(slot of root(x), slot of root(y), level)
  constexpr int kBatch = 8;
#pragma unroll
  for (int k0 = 0; k0 < kLdsPer; k0 += kBatch) {
    int2 e[kBatch];
    int32_t fa[kBatch], fb[kBatch], ga[kBatch], gb[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int g = tid + (k0 + j) * kTileThreads;
      e[j] = make_int2(-1, -1);
      if (g < total) {
        const int2 x = edge_at(g);
        const int lv = cross_level(x.x, x.y);
        // (a group block reading the full list keeps its own group's edges)
        if (lv >= lo && lv < hi && (!grp || !from_list || (x.x >> (kTileShift + group_log)) == (int32_t)blockIdx.x))
          e[j] = x;
      }
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      fa[j] = e[j].x >= 0 ? cc[e[j].x] : 0;
      fb[j] = e[j].x >= 0 ? cc[e[j].y] : 0;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      ga[j] = e[j].x >= 0 ? cc[fa[j]] : 0;
      gb[j] = e[j].x >= 0 ? cc[fb[j]] : 0;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      sab[k0 + j] = ~0u;
      if (e[j].x >= 0) {
        const int32_t ra = ga[j] == fa[j] ? fa[j] : find_root(ga[j], cc);
        const int32_t rb = gb[j] == fb[j] ? fb[j] : find_root(gb[j], cc);
        if (ra < own_lo || ra > own_hi || rb < own_lo || rb > own_hi) {
          s_fail = 1;                     // a root owned by another group
        } else if (ra != rb) {
          const int sa = lds_slot(ra, keys), sb = lds_slot(rb, keys);
          if (sa < 0 || sb < 0) s_fail = 1;
          else sab[k0 + j] = pack_sab(sa, sb, 0);
        }
      }
    }
  }
  __syncthreads();
  if (s_fail) {
    if (tid == 0) counters[kCntCrossOverflow] = 1;
    return;
  }
  // all levels in one pass: in LDS the order of the unions only changes
  // which spanning edges are chosen, and path halving keeps the finds short
#pragma unroll
  for (int k = 0; k < kLdsPer; ++k) {
    const uint32_t v = sab[k];
    if (v != ~0u)
      lds_union((int)(v & 0x3fff), (int)((v >> 14) & 0x3fff), tid + k * kTileThreads, keys, par,
                s_hooks, &s_nhooks);
  }
  __syncthreads();
  // Every hooked root points straight at its final root and records the kept
  // edge that hooked it; the unions listed the hooked slots, one thread each
  // finishes them, so their edge lookups and global writes proceed in parallel.
  const int nh = s_nhooks;
  for (int r = tid; r < nh; r += kTileThreads) {
    const int hi = s_hooks[r];
    const int g = (par[hi] >> 14) - 1;
    const int32_t key = keys[hi];
    const int32_t root = keys[lds_find_rec(hi, par)];
    const int2 e = edge_at(g);
    store_agent(&cc[key], root);
    tu[key] = e.x;
    tv[key] = e.y;
    if (head) link_slot(key, e.x, e.y, head, next);
  }
  if (all && tid == 0) counters[kCntCrossDone] = 1;   // (visible to the next kernel)
  block_release_device();
}

// Global-memory hooking after the LDS merges, in one launch.  Only when an LDS
// merge raised the flag (its kept edges or roots did not fit), every kept
// cross edge is hooked here by compare-and-swap, the tiles' kept edges spread
// over the whole grid in no particular order (hooking is correct in any order;
// on the graphs that get here -- ids without locality, millions of kept edges
// -- one workgroup per level or group would serialise the work).  The heavy-
// vertex chunks are hooked by the same grid, side by side.
template <class OffT>
__global__ __launch_bounds__(kTileThreads) void k_late_hooks(
    const int64_t *__restrict__ region_of, const int2 *__restrict__ cross,
    const int32_t *__restrict__ tile_cross, int tiles, int slices, const OffT *__restrict__ off,
    const int32_t *__restrict__ cols, const int64_t *chunks, int64_t chunk_cap, int32_t *cc,
    int32_t *tu, int32_t *tv, int32_t *counters, int32_t *head, int32_t *next) {
  const int tid = threadIdx.x;
  bool hooked = false;
  if (counters[kCntCrossOverflow]) {   // block-uniform
    // tile b's kept edges by blocks b*slices .. (b+1)*slices-1 (mod the grid)
    for (int64_t w = blockIdx.x; w < (int64_t)tiles * slices; w += gridDim.x) {
      const int64_t b = w / slices;
      const int part = (int)(w % slices);
      const int kept = kept_count(tile_cross[b]);
      const int64_t region = region_of[b];
      for (int i = part * kTileThreads + tid; i < kept; i += slices * kTileThreads) {
        const int2 e = cross[region + i];
        hook_edge<true>(e.x, e.y, cc, tu, tv, head, next);
      }
      hooked = true;
    }
  }
  int64_t nc = counters[kCntChunks];
  if (nc > chunk_cap) nc = chunk_cap;
  for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const int64_t w = chunks[c];
    const int32_t src = (int32_t)(w >> 32);
    const int64_t k = w & 0xffffffffll;
    const int64_t b = (int64_t)off[src] + k * kChunk;
    int64_t e = (int64_t)off[src + 1];
    if (e > b + kChunk) e = b + kChunk;
    for (int64_t a = b + tid; a < e; a += kTileThreads) {
      const int32_t dst = cols[a];
      if (dst < src) hook_edge<true>(src, dst, cc, tu, tv, head, next);
    }
    hooked = true;
  }
  if (hooked) block_release_device();   // block-uniform: only blocks that hooked
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
  wave_release_device();
}

// Final pointer jumping: every vertex points at its root (= min id of its
// component).  Also resets the per-vertex arrays the rooting stage needs.
template <int B>
__global__ __launch_bounds__(B) void k_compress(int64_t n, int32_t *cc, int32_t *comp_root,
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
  int64_t heavy = ctx->opt.heavy_degree < 1 ? 1 : ctx->opt.heavy_degree;
  if (heavy > kTileLightMax) heavy = kTileLightMax;   // the tile pass takes no larger degree
  return (size_t)(nnz / kChunk + nnz / (heavy + 1) + 2);
}

rst_status enqueue_reset_counters(rst_ctx *ctx, int32_t *counters, int32_t root) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, ctx->stream, counters, root);
  RST_HIP(hipGetLastError());
  return RST_OK;
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
// tile_cross buffer: int32 counts, int64 region starts, int32 level ranges,
// then the compact lists of kept cross edges, all levels and the top levels
// (int2 [kLdsEdges] each)
size_t hook_tile_words(int64_t n) {
  const size_t tc = hook_tile_count(n), even = (tc + 1) & ~size_t(1);
  return even + 2 * tc + even + 4 * (size_t)kLdsEdges;
}

static rst_status launch_cross(rst_ctx *ctx, unsigned tiles, int levels,
                               const int64_t *region_of, int2 *cross, int32_t *tile_cross,
                               const int32_t *tile_lvl, int2 *kept_list, ForestBufs &f) {
  if (levels == 0) return RST_OK;       // one tile: no cross edges
  RST_KMARK(ctx, RST_KERNEL_CROSS, 0);
  // levels below `split` are merged per group of 2^split tiles (one workgroup
  // each), the rest by one workgroup
  int split = levels <= 3 ? 0 : levels / 2;
  if (split > 10) split = 10;
  // flat tiles are split over several blocks when there are fewer tiles than
  // two per CU (every extra block is dispatched, and leaves at once, for every
  // tile that is not flat)
  const unsigned target = (unsigned)(ctx->num_cus * 2);
  unsigned slices = (target + tiles - 1) / tiles;
  slices = slices < 1 ? 1 : (slices > 64 ? 64 : slices);
  hipLaunchKernelGGL(k_cross_dedupe, dim3(tiles * slices), dim3(kTileThreads), 0, ctx->stream,
                     region_of, cross, tile_cross, (int)slices, f.cc, f.tu, f.tv, f.counters,
                     kept_list, split, f.head, f.next);
  RST_HIP(hipGetLastError());
  const unsigned groups = (tiles + (1u << split) - 1) >> split;
  if (split > 0) {
    // per group of 2^split tiles below `split` (or, with few kept edges, all
    // levels in block 0), then one block for the levels above
    hipLaunchKernelGGL(k_cross_lds<true>, dim3(groups), dim3(kTileThreads), 0, ctx->stream,
                       region_of, cross, tile_cross, kept_list, (int)tiles, 0, split, split,
                       levels, f.cc, f.tu, f.tv, f.counters, f.head, f.next);
    RST_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_cross_lds<false>, dim3(1), dim3(kTileThreads), 0, ctx->stream, region_of,
                     cross, tile_cross, kept_list, (int)tiles, split, levels, levels, levels, f.cc,
                     f.tu, f.tv, f.counters, f.head, f.next);
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_CROSS, 1);
  return RST_OK;
}

// The global-memory fallback of the cross merges (active only when an LDS
// merge raised its flag) and the heavy chunks, in one launch.
template <class OffT>
static rst_status launch_late_hooks(rst_ctx *ctx, unsigned tiles, int levels,
                                    const int64_t *region_of, const int2 *cross,
                                    const int32_t *tile_cross, const OffT *off,
                                    const int32_t *cols, const int64_t *chunks, int64_t chunk_cap,
                                    ForestBufs &f) {
  const unsigned grid = (unsigned)(ctx->num_cus * 2);
  unsigned slices = (grid + tiles - 1) / tiles;
  slices = slices < 1 ? 1 : (slices > 64 ? 64 : slices);
  RST_KMARK(ctx, RST_KERNEL_LATE_HOOKS, 0);
  hipLaunchKernelGGL(k_late_hooks<OffT>, dim3(grid), dim3(kTileThreads), 0, ctx->stream, region_of,
                     cross, tile_cross, levels == 0 ? 0 : (int)tiles, (int)slices, off, cols, chunks,
                     chunk_cap, f.cc, f.tu, f.tv, f.counters, f.head, f.next);
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_LATE_HOOKS, 1);
  return RST_OK;
}

rst_status enqueue_hook_csr(rst_ctx *ctx, const rst_csr *g, ForestBufs &f, int64_t *chunks,
                            int64_t chunk_cap, int2 *cross, int32_t *tile_cross) {
  const size_t tc = hook_tile_count(g->n);
  int64_t *region_of = reinterpret_cast<int64_t *>(tile_cross + ((tc + 1) & ~size_t(1)));
  int32_t *tile_lvl = reinterpret_cast<int32_t *>(region_of + tc);
  int2 *kept_list = reinterpret_cast<int2 *>(tile_lvl + ((tc + 1) & ~size_t(1)));
  const int64_t n = g->n;
  const unsigned tiles = grid_for(n, kTile);
  // bit 0: 16-byte loads of cols allowed, bit 1: of the offsets
  const int vec_cols = (((uintptr_t)g->cols & 15) == 0 ? 1 : 0) | (((uintptr_t)g->offsets & 15) == 0 ? 2 : 0);
  int levels = 0;
  while ((1u << levels) < tiles) ++levels;
  if (g->offset_bytes == 4) {
    const int32_t *off = (const int32_t *)g->offsets;
    RST_KMARK(ctx, RST_KERNEL_HOOK_TILE, 0);
    hipLaunchKernelGGL(k_hook_tile<int32_t>, dim3(tiles), dim3(kTileThreads), 0, ctx->stream, n,
                       off, g->cols, f.cc, f.tu, f.tv, cross, tile_cross, tile_lvl, region_of,
                       f.counters, chunks, chunk_cap, ctx->opt.heavy_degree, f.vmask, f.head,
                       f.next, vec_cols, f.gsel);
    RST_HIP(hipGetLastError());
    RST_KMARK(ctx, RST_KERNEL_HOOK_TILE, 1);
    RST_TRY(launch_cross(ctx, tiles, levels, region_of, cross, tile_cross, tile_lvl, kept_list, f));
    RST_TRY(launch_late_hooks(ctx, tiles, levels, region_of, cross, tile_cross, off, g->cols,
                              chunks, chunk_cap, f));
  } else {
    const int64_t *off = (const int64_t *)g->offsets;
    RST_KMARK(ctx, RST_KERNEL_HOOK_TILE, 0);
    hipLaunchKernelGGL(k_hook_tile<int64_t>, dim3(tiles), dim3(kTileThreads), 0, ctx->stream, n,
                       off, g->cols, f.cc, f.tu, f.tv, cross, tile_cross, tile_lvl, region_of,
                       f.counters, chunks, chunk_cap, ctx->opt.heavy_degree, f.vmask, f.head,
                       f.next, vec_cols, f.gsel);
    RST_HIP(hipGetLastError());
    RST_KMARK(ctx, RST_KERNEL_HOOK_TILE, 1);
    RST_TRY(launch_cross(ctx, tiles, levels, region_of, cross, tile_cross, tile_lvl, kept_list, f));
    RST_TRY(launch_late_hooks(ctx, tiles, levels, region_of, cross, tile_cross, off, g->cols,
                              chunks, chunk_cap, f));
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
  RST_SWEEP(ctx, k_compress, n, n, cc, comp_root, head);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

}  // namespace rst
