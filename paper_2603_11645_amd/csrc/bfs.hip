// bfs.hip -- level-synchronous breadth-first search (Sec. III-A), the baseline.
//
// A level: every frontier vertex offers all its arcs, an unvisited neighbour
// is claimed (its level set to L+1, the claiming source becomes its parent)
// and appended to the next frontier.  Wide levels (large frontiers) follow
// the edge-centric idea of Merrill et al. (Sec. II): a workgroup takes 1024
// frontier vertices, scans their degrees in LDS and walks the union of their
// arcs with unit stride, so a thread handles arcs, not vertices; claims are
// compare-and-swaps on the level; vertices above a degree threshold go to a
// separate "heavy" frontier, each expanded by a whole workgroup;
// appends use one atomic per wavefront (ballot + mbcnt).  Narrow levels
// (small frontiers, i.e. almost every level of a high-diameter graph) run
// many to a launch in one workgroup (k_bfs_step), so the cost of a level is
// two dependent rounds of memory accesses plus a workgroup barrier instead
// of a kernel launch.
//
// Frontier sizes and the level reached live in device memory, so the host
// enqueues steps back to back and only reads them once per batch; a step
// whose input frontier is empty returns at once.  Counts rotate over three
// slots: level L reads slot L%3, appends to slot (L+1)%3 and clears slot
// (L+2)%3, which the level after it appends to.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

__global__ void k_bfs_reset(int64_t n, int32_t *level, int32_t *parent, int32_t *cnt) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    level[v] = -1;
    if (parent) parent[v] = -1;
  }
  if (v < kBfsCntWords) cnt[v] = 0;
}

// Arcs of a level's light frontier, counted exactly up to kBsArcsCount and
// left above it once passed (adds stop there, so the count cannot overflow):
// a step knows before it starts whether the level fits the narrow mode.
constexpr int kBsArcsCount = 4096;   // equals kBsArcs below

template <class OffT>
__device__ __forceinline__ void bfs_enqueue(bool win, int32_t w, const OffT *off, int heavy_deg,
                                            int32_t *qout, int32_t *hout, int32_t *cout,
                                            int32_t *arcs, int64_t heavy_cap, int32_t *counters) {
  bool heavy = false;
  int64_t deg = 0;
  if (win) {
    deg = (int64_t)(off[w + 1] - off[w]);
    heavy = deg > heavy_deg;
  }
  const bool light = win && !heavy;
  const int sl = wave_append(light, &cout[0]);
  if (light) qout[sl] = w;
  const int sh = wave_append(win && heavy, &cout[1]);
  if (win && heavy && sh < heavy_cap) hout[sh] = w;
  wave_count(win, &counters[kCntBfsReached]);
  // wave sum of the light degrees (each clamped), one add per wave
  int d = light ? (int)(deg > kBsArcsCount ? kBsArcsCount + 1 : deg) : 0;
  for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
  if ((threadIdx.x & 63) == 0 && d > 0 && *reinterpret_cast<volatile int32_t *>(arcs) <= kBsArcsCount)
    atomicAdd(arcs, d > kBsArcsCount ? kBsArcsCount + 1 : d);
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
  bfs_enqueue<OffT>(win, r, off, heavy_deg, q0, h0, cnt0, cnt0 + kBfsArcsWord, heavy_cap,
                    counters);
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
    store_agent(&level[v], 0);
    parent[v] = (int32_t)v;
    win = true;
  }
  bfs_enqueue<OffT>(win, (int32_t)v, off, heavy_deg, q0, h0, cnt0, cnt0 + kBfsArcsWord,
                    heavy_cap, counters);
}

// ---------------------------------------------------------------------------
// One level step.  A launch reads the level L it starts at from the state
// words (state[par]) and leaves the level it reached in state[par ^ 1], so
// that the host can enqueue steps without knowing how far each one got.
//
// Wide mode (the frontier holds heavy vertices or more than kBsMax): every
// workgroup takes its share of the frontier and the level is expanded once,
// as described at the top of this file.
//
// Narrow mode (a small frontier, which on high-diameter graphs is every
// level): workgroup 0 alone runs level after level with only workgroup
// barriers between them, the frontier and each vertex's arc range kept in
// LDS; the other workgroups leave at once.  A level claims its new vertices
// by a plain store of their level after deduplicating them in an LDS hash
// (one workgroup sees every write of the level), and the arc range of a new
// vertex is loaded together with its level, so a level costs two dependent
// rounds of global loads (its arcs' neighbour ids, then their levels and arc
// ranges).  Narrow mode stops when the frontier outgrows LDS or holds a heavy
// vertex (the frontier is then left in the global queues for a wide step),
// when a level would expand more than kBsArcs arcs (the next step is then
// forced wide), after kBsBudget levels, at level_stop, or when the search is
// done.
// ---------------------------------------------------------------------------
constexpr int kBfsThreads = 1024;
constexpr int kBsMax = 2048;           // frontier vertices held in LDS (narrow mode)
constexpr int kBsArcs = kBsArcsCount;  // arcs one narrow level may expand
constexpr int kBsHash = 8192;          // deduplication slots, > 2 * kBsArcs: never full
constexpr int kBsBudget = 1 << 18;     // narrow levels per launch
static_assert(kBsHash >= 2 * kBsArcs && kBsMax == 2 * kBfsThreads, "narrow-mode sizes");

template <class OffT>
struct BfsSmem {
  union {
    struct {
      int32_t v[2][kBsMax];    // frontier vertices (current, next)
      OffT b[2][kBsMax];       // their first arc
      int32_t d[2][kBsMax];    // their degree (capped at kBsArcs + 1)
      int32_t scan[kBsMax + 1];
      int32_t hash[kBsHash];
    } nar;
    struct {
      int scan[kBfsThreads + 1];
      OffT beg[kBfsThreads];
      int32_t src[kBfsThreads];
      int32_t st_l[kBfsThreads];   // vertices claimed by one round, light / heavy
      int32_t st_h[kBfsThreads];
      int nl, nh, base_l, base_h;
    } wide;
  };
  int wave[kBfsThreads / kWave];
  int nn;
};

__device__ __forceinline__ uint32_t bfs_hash(int32_t w) {
  return ((uint32_t)w * 0x9E3779B1u) >> (32 - 13);   // 13 bits: kBsHash slots
}
static_assert(kBsHash == 1 << 13, "bfs_hash gives 13 bits");

// state: [0..1] level by launch parity, [2..3] "next step wide" by parity
template <class OffT>
__global__ __launch_bounds__(kBfsThreads) void k_bfs_step(
    int par, const OffT *__restrict__ off, const int32_t *__restrict__ cols, int32_t *level,
    int32_t *parent, int32_t *q0, int32_t *q1, int32_t *h0, int32_t *h1, int32_t *cnt,
    int32_t *state, int64_t heavy_cap, int32_t *counters, int heavy_deg, int32_t level_stop) {
  __shared__ BfsSmem<OffT> sh;
  const int t = threadIdx.x;
  int32_t L = state[par];
  const bool force_wide = state[2 + par] != 0;
  int nl = cnt[2 * (L % 3)];
  int nh = cnt[2 * (L % 3) + 1];
  const int arcs_l = cnt[kBfsArcsWord + L % 3];
  if (nh > heavy_cap) nh = (int)heavy_cap;
  if (L >= level_stop || nl + nh == 0) {
    if (blockIdx.x == 0 && t == 0) { state[par ^ 1] = L; state[2 + (par ^ 1)] = 0; }
    return;
  }
  if (nh == 0 && nl <= kBsMax && arcs_l <= kBsArcs && !force_wide) {
    // ------------------------------------------------------------ narrow
    if (blockIdx.x != 0) return;
    const int32_t *qin = (L & 1) ? q1 : q0;
    for (int i = t; i < nl; i += kBfsThreads) {
      const int32_t u = qin[i];
      const OffT b = off[u], e = off[u + 1];
      sh.nar.v[0][i] = u;
      sh.nar.b[0][i] = b;
      sh.nar.d[0][i] = (int32_t)((e - b) > (OffT)kBsArcs ? (OffT)(kBsArcs + 1) : (e - b));
    }
    int c = 0, nf = nl;
    bool wide_next = false, spill = false;   // spill: the frontier is only in LDS
    for (int it = 0; it < kBsBudget; ++it) {
      __syncthreads();
      const int i0 = 2 * t;
      const int d0 = i0 < nf ? sh.nar.d[c][i0] : 0;
      const int d1 = i0 + 1 < nf ? sh.nar.d[c][i0 + 1] : 0;
      int tot;
      const int ex = block_excl_scan<kBfsThreads>(d0 + d1, sh.wave, &tot);
      if (tot > kBsArcs) { wide_next = true; break; }   // uniform: leave this level to a wide step
      if (i0 < nf) sh.nar.scan[i0] = ex;
      if (i0 + 1 < nf) sh.nar.scan[i0 + 1] = ex + d0;
      for (int j = t; j < kBsHash; j += kBfsThreads) sh.nar.hash[j] = -1;
      int32_t *cnext = cnt + 2 * ((L + 1) % 3);
      if (t == 0) {
        sh.nar.scan[nf] = tot;
        sh.nn = 0;
        cnext[1] = 0;                            // heavy appends of the next level
        counters[kCntBfsLast] = L;
      }
      __syncthreads();
      const int32_t nxl = L + 1;
      int32_t *qout = (nxl & 1) ? q1 : q0;
      int32_t *hout = (nxl & 1) ? h1 : h0;
      for (int k0 = 0; k0 < tot; k0 += kBfsThreads) {
        const int k = k0 + t;
        bool claim = false;
        int32_t w = -1, u = -1;
        OffT wb = 0, we = 0;
        if (k < tot) {
          const int j = lds_upper_search(sh.nar.scan, nf, k);
          u = sh.nar.v[c][j];
          w = cols[sh.nar.b[c][j] + (OffT)(k - sh.nar.scan[j])];
          const int32_t lw = level[w];
          wb = off[w];
          we = off[w + 1];
          if (lw == -1) {
            uint32_t h = bfs_hash(w);
            while (true) {   // at most kBsArcs keys in kBsHash slots: a free one exists
              const int32_t old = atomicCAS(&sh.nar.hash[h], -1, w);
              if (old == -1) { claim = true; break; }
              if (old == w) break;
              h = (h + 1) & (kBsHash - 1);
            }
          }
        }
        if (claim) {
          store_agent(&level[w], nxl);   // wide steps on other XCDs may compare-and-swap it
          if (parent) parent[w] = u;
        }
        const bool heavy = claim && (int64_t)(we - wb) > heavy_deg;
        const bool light = claim && !heavy;
        const int sl = wave_append(light, &sh.nn);
        if (light) {
          if (sl < kBsMax) {
            sh.nar.v[c ^ 1][sl] = w;
            sh.nar.b[c ^ 1][sl] = wb;
            sh.nar.d[c ^ 1][sl] = (int32_t)((we - wb) > (OffT)kBsArcs ? (OffT)(kBsArcs + 1) : (we - wb));
          } else {
            qout[sl] = w;      // beyond LDS: straight to the global queue
          }
        }
        const int shv = wave_append(heavy, &cnext[1]);
        if (heavy && shv < heavy_cap) hout[shv] = w;
        wave_count(claim, &counters[kCntBfsReached]);
      }
      __syncthreads();
      const int nn = sh.nn;
      const int nhv = __hip_atomic_load(&cnext[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      L = nxl;
      c ^= 1;
      nf = nn;
      spill = true;
      if (nn == 0 && nhv == 0) { spill = false; break; }     // search done
      if (nn > kBsMax || nhv > 0 || L >= level_stop) break;
    }
    __syncthreads();
    // leave the frontier of level L in the global queues for the next step
    if (spill) {
      int32_t *q = (L & 1) ? q1 : q0;
      const int m = nf < kBsMax ? nf : kBsMax;
      for (int i = t; i < m; i += kBfsThreads) q[i] = sh.nar.v[c][i];
    }
    // arcs of that frontier (only needed when it fits LDS)
    int ad = 0;
    if (nf <= kBsMax)
      for (int i = t; i < nf; i += kBfsThreads) ad += sh.nar.d[c][i];
    int atot;
    (void)block_excl_scan<kBfsThreads>(ad, sh.wave, &atot);
    if (t == 0) {
      cnt[2 * (L % 3)] = nf;              // light count (heavy count already there)
      cnt[kBfsArcsWord + L % 3] = nf <= kBsMax ? atot : kBsArcs + 1;
      cnt[2 * ((L + 1) % 3)] = 0;         // the next step appends here
      cnt[2 * ((L + 1) % 3) + 1] = 0;
      cnt[kBfsArcsWord + (L + 1) % 3] = 0;
      state[par ^ 1] = L;
      state[2 + (par ^ 1)] = wide_next ? 1 : 0;
    }
    return;
  }
  // -------------------------------------------------------------- wide
  const int nxt = (L + 1) % 3, clr = (L + 2) % 3;
  const int32_t *qin = (L & 1) ? q1 : q0;
  const int32_t *hin = (L & 1) ? h1 : h0;
  int32_t *qout = (L & 1) ? q0 : q1;
  int32_t *hout = (L & 1) ? h0 : h1;
  int32_t *cout = cnt + 2 * nxt;
  int32_t *aout = cnt + kBfsArcsWord + nxt;
  if (blockIdx.x == 0 && t < 2) cnt[2 * clr + t] = 0;
  if (blockIdx.x == 0 && t == 2) cnt[kBfsArcsWord + clr] = 0;
  if (blockIdx.x == 0 && t == 0) {
    counters[kCntBfsLast] = L;
    state[par ^ 1] = L + 1;
    state[2 + (par ^ 1)] = 0;
  }
  if (t == 0) { sh.wide.nl = 0; sh.wide.nh = 0; }
  const int32_t next_level = L + 1;
  // Claimed vertices are staged in LDS (one LDS atomic per wave) and appended
  // to the next frontier by one global atomic per workgroup and round of 1024
  // arcs; the reached and arc counts go out once per workgroup at the end.
  // (One global atomic per wave on the same few counters serialised the wide
  // levels of power-law graphs: milliseconds per level.)
  int reached = 0, arcs_sum = 0;
  auto emit = [&](bool win, int32_t w) {   // all threads of the workgroup
    int64_t deg = 0;
    bool heavy = false;
    if (win) {
      deg = (int64_t)(off[w + 1] - off[w]);
      heavy = deg > heavy_deg;
    }
    const bool light = win && !heavy;
    const int sl = wave_append(light, &sh.wide.nl);
    if (light) sh.wide.st_l[sl] = w;
    const int sv = wave_append(win && heavy, &sh.wide.nh);
    if (win && heavy) sh.wide.st_h[sv] = w;
    reached += win ? 1 : 0;
    if (light && arcs_sum <= kBsArcsCount)
      arcs_sum += (int)(deg > kBsArcsCount ? kBsArcsCount + 1 : deg);
    __syncthreads();
    if (t == 0) {
      sh.wide.base_l = sh.wide.nl ? atomicAdd(&cout[0], sh.wide.nl) : 0;
      sh.wide.base_h = sh.wide.nh ? atomicAdd(&cout[1], sh.wide.nh) : 0;
    }
    __syncthreads();
    const int na = sh.wide.nl, nb = sh.wide.nh, ba = sh.wide.base_l, bb = sh.wide.base_h;
    for (int i = t; i < na; i += kBfsThreads) qout[ba + i] = sh.wide.st_l[i];
    for (int i = t; i < nb; i += kBfsThreads)
      if (bb + i < heavy_cap) hout[bb + i] = sh.wide.st_h[i];
    __syncthreads();
    if (t == 0) { sh.wide.nl = 0; sh.wide.nh = 0; }
    __syncthreads();
  };

  for (int64_t c0 = (int64_t)blockIdx.x * kBfsThreads; c0 < nl;
       c0 += (int64_t)gridDim.x * kBfsThreads) {
    const int64_t i = c0 + t;
    int deg = 0;
    OffT beg = 0;
    int32_t u = -1;
    if (i < nl) {
      u = qin[i];
      beg = off[u];
      deg = (int)(off[u + 1] - beg);
    }
    sh.wide.beg[t] = beg;
    sh.wide.src[t] = u;
    int total;
    const int excl = block_excl_scan<kBfsThreads>(deg, sh.wave, &total);
    sh.wide.scan[t] = excl;
    if (t == kBfsThreads - 1) sh.wide.scan[kBfsThreads] = excl + deg;
    __syncthreads();
    for (int b = 0; b < total; b += kBfsThreads) {
      const int k = b + t;
      int32_t w = -1, src = -1;
      if (k < total) {
        const int j = lds_upper_search(sh.wide.scan, kBfsThreads, k);
        src = sh.wide.src[j];
        w = cols[(int64_t)sh.wide.beg[j] + (k - sh.wide.scan[j])];
      }
      bool win = false;
      if (w >= 0 && level[w] == -1 && atomicCAS(&level[w], -1, next_level) == -1) {
        win = true;
        if (parent) parent[w] = src;
      }
      emit(win, w);
    }
    __syncthreads();
  }

  // heavy vertices: a workgroup takes whole vertices in turn (every workgroup
  // walking every heavy vertex's range cost one round trip per vertex per
  // workgroup, milliseconds per level on power-law graphs)
  for (int hi = blockIdx.x; hi < nh; hi += gridDim.x) {
    const int32_t u = hin[hi];
    const int64_t b = (int64_t)off[u], e = (int64_t)off[u + 1];
    for (int64_t a0 = b; a0 < e; a0 += kBfsThreads) {
      const int64_t a = a0 + t;
      const int32_t w = a < e ? cols[a] : -1;
      bool win = false;
      if (w >= 0 && level[w] == -1 && atomicCAS(&level[w], -1, next_level) == -1) {
        win = true;
        if (parent) parent[w] = u;
      }
      emit(win, w);
    }
  }
  int block_reached, block_arcs;
  (void)block_excl_scan<kBfsThreads>(reached, sh.wave, &block_reached);
  (void)block_excl_scan<kBfsThreads>(arcs_sum, sh.wave, &block_arcs);
  if (t == 0) {
    if (block_reached) atomicAdd(&counters[kCntBfsReached], block_reached);
    if (block_arcs > 0 && *reinterpret_cast<volatile int32_t *>(aout) <= kBsArcsCount)
      atomicAdd(aout, block_arcs > kBsArcsCount ? kBsArcsCount + 1 : block_arcs);
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
  const int64_t items = n > kBfsCntWords ? n : kBfsCntWords;
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
  // counts of slot 0 and the level state must start from zero for this new frontier
  RST_TRY(enqueue_fill(ctx, b.cnt, kBfsCntWords, 0));
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
static rst_status launch_step(rst_ctx *ctx, const rst_csr *g, int par, unsigned grid,
                              int32_t *level, int32_t *parent, BfsBufs &b, int32_t *counters,
                              int32_t level_stop) {
  hipLaunchKernelGGL(k_bfs_step<OffT>, dim3(grid), dim3(kBfsThreads), 0, ctx->stream, par,
                     (const OffT *)g->offsets, g->cols, level, parent, b.q[0], b.q[1], b.h[0],
                     b.h[1], b.cnt, b.cnt + kBfsStateWord, b.heavy_cap, counters,
                     ctx->opt.bfs_heavy_degree, level_stop);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status bfs_enqueue_steps(rst_ctx *ctx, const rst_csr *g, int32_t *level, int32_t *parent,
                             BfsBufs &b, int32_t *counters, int64_t steps, int64_t max_levels) {
  const unsigned grid = ctx->opt.bfs_grid > 0 ? (unsigned)ctx->opt.bfs_grid
                                              : (unsigned)ctx->num_cus;
  const int32_t level_stop = max_levels >= 0 && max_levels < 0x7fffffff ? (int32_t)max_levels
                                                                         : 0x7fffffff;
  steps += steps & 1;   // an even count leaves the level in state[0]
  for (int64_t k = 0; k < steps; ++k) {
    const int par = (int)(k & 1);
    if (g->offset_bytes == 4)
      RST_TRY(launch_step<int32_t>(ctx, g, par, grid, level, parent, b, counters, level_stop));
    else
      RST_TRY(launch_step<int64_t>(ctx, g, par, grid, level, parent, b, counters, level_stop));
  }
  return RST_OK;
}

rst_status bfs_run_levels(rst_ctx *ctx, const rst_csr *g, int32_t *level, int32_t *parent,
                          BfsBufs &b, int32_t *counters, int64_t *levels_out, int64_t max_levels) {
  const int per_sync = ctx->opt.bfs_levels_per_sync < 1 ? 1 : ctx->opt.bfs_levels_per_sync;
  // wide steps: one workgroup of 1024 per CU unless set
  const unsigned grid = ctx->opt.bfs_grid > 0 ? (unsigned)ctx->opt.bfs_grid
                                              : (unsigned)ctx->num_cus;
  const int32_t level_stop = max_levels >= 0 && max_levels < 0x7fffffff ? (int32_t)max_levels
                                                                         : 0x7fffffff;
  int par = 0;           // the level starts in state[0] (zeroed with the counts)
  int64_t steps = 0;
  for (;;) {
    for (int k = 0; k < per_sync; ++k, ++steps) {
      if (g->offset_bytes == 4)
        RST_TRY(launch_step<int32_t>(ctx, g, par, grid, level, parent, b, counters, level_stop));
      else
        RST_TRY(launch_step<int64_t>(ctx, g, par, grid, level, parent, b, counters, level_stop));
      par ^= 1;
    }
    // the level reached and its frontier counts
    RST_HIP(hipMemcpyAsync(ctx->host_pinned, b.cnt, kBfsCntWords * sizeof(int32_t),
                           hipMemcpyDeviceToHost, ctx->stream));
    RST_HIP(hipStreamSynchronize(ctx->stream));
    const int32_t L = ctx->host_pinned[kBfsStateWord + par];
    if (ctx->host_pinned[2 * (L % 3)] == 0 && ctx->host_pinned[2 * (L % 3) + 1] == 0) break;
    if (L >= level_stop) break;   // capped search (depth probes)
    if (steps > 2 * (g->n + per_sync) + 64) return RST_E_DEVICE;   // cannot happen for a valid CSR
  }
  RST_HIP(hipMemcpyAsync(ctx->host_pinned + 2, counters + kCntBfsLast, sizeof(int32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  if (levels_out) *levels_out = ctx->host_pinned[2];
  return RST_OK;
}

}  // namespace rst
