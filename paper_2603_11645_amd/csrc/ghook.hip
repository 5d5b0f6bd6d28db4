// ghook.hip -- hooking in global memory for graphs whose vertex ids carry no
// locality (random labels: R-MAT, permuted meshes, long chains).  Same hooking
// rule as hook.hip (Sec. III-B: the larger root is linked under the smaller by
// compare-and-swap, the edge behind every successful hook recorded at the
// hooked root, Sec. I) and the same Euler arc lists (link_slot, inside the
// hook: a separate pass over the slots afterwards took longer, its exchanges
// no longer overlapping the hooks' other memory accesses), but no vertex
// tiles: on such graphs almost every edge crosses tiles, so the tile pass and
// the cross-tile merges only add work.
//
// Sec. III-B leaves the order of hooking open.  The sweep here follows the
// sampling idea of Afforest (Sutton et al.): a vertex first hooks along K of
// its arcs, which on graphs of average degree well above 2 already joins most
// vertices into one dominant tree; one workgroup then finds the most frequent
// root in a sample of vertices.  The full sweep visits the arcs again, and a
// vertex that is already in the dominant tree offers none: the arcs it skips
// lead either into the dominant tree too or to a vertex outside it, which
// offers the reverse arc itself (the CSR is symmetric).  Without a dominant
// tree (chains, meshes: no sample root holds half the sample) each edge is
// visited once instead, from its larger end, after a first pass without
// finds: every vertex hooks to the smallest of the first kGhMinArcs
// neighbours when that one is smaller than itself (pointers to smaller ids
// cannot close a cycle, so this is a forest of valid hooks, taken reading
// only the vertex's own arcs); on a chain with random ids it hooks two
// thirds of the vertices, and the sweep skips those edges.
#include "rst_internal.h"
#include "device_common.h"
#include "unionfind.h"

namespace rst {

constexpr int kGhThreads = 1024;      // vertices per workgroup of the arc sweep
constexpr int kGhSampleThreads = 1024;
constexpr int kGhSamplePer = 4;       // sampled vertices per thread (giant, probe)
constexpr int kGhHash = 8192;         // LDS hash slots of the root count
constexpr int kGhTileShift = 13;      // the tile pass's tile: 8192 consecutive ids
constexpr int kGhMinArcs = 16;        // arcs the first pass looks at per vertex

// counter-based sample index (splitmix64 finaliser of seed ^ i)
__device__ __forceinline__ uint64_t gh_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// root of x without writes (cc[y] <= y, equality at roots)
__device__ __forceinline__ int32_t gh_root(int32_t x, const int32_t *cc) {
  int32_t r = x, nx;
  while (r > (nx = cc[r])) r = nx;
  return r;
}

// Every vertex its own tree, every slot empty, every arc list empty.
template <int B>
__global__ __launch_bounds__(B) void k_gh_init(int64_t n, int32_t *cc, int32_t *tu, int32_t *tv,
                                               int32_t *head) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  store_agent(&cc[v], (int32_t)v);
  tu[v] = -1;
  tv[v] = -1;
  if (head) store_agent(&head[v], -1);
}

// The first pass without a dominant tree: v (still a root, fresh from
// k_gh_init) hooks to m, the smallest of its first kGhMinArcs neighbours, when
// m < v; the edge (v, m) goes to slot v.  Only v's own word changes, so no
// compare-and-swap is needed; the sweep after it reads the words (agent-scope
// stores) and puts the slot's arcs onto the lists (there the exchanges
// overlap the sweep's finds; here they cost the pass most of its time).
template <class OffT>
__global__ __launch_bounds__(kBlock) void k_gh_minhook(int64_t n, const OffT *__restrict__ off,
                                                       const int32_t *__restrict__ cols,
                                                       const uint8_t *__restrict__ vmask,
                                                       int32_t *cc, int32_t *tu, int32_t *tv) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || (vmask && vmask[v])) return;
  const OffT b = off[v], e = off[v + 1];
  const OffT last = e - b > kGhMinArcs ? b + kGhMinArcs : e;
  int32_t m = (int32_t)v;
  for (OffT a = b; a < last; ++a) {
    const int32_t w = cols[a];
    if (w >= 0 && w < m) m = w;
  }
  if (m == (int32_t)v) return;
  store_agent(&cc[v], m);
  tu[v] = (int32_t)v;
  tv[v] = m;
}

// Each vertex hooks along K of its arcs (all of them when it has at most K),
// taken at pseudo-random positions: on power-law graphs with sorted neighbour
// lists the first arcs of almost every vertex lead to the same few hubs.
// Every hook puts an arc at the front of both ends' lists; the arcs into the
// sampled neighbours' lists are pushed wave by wave with wave_push_front,
// since many lanes of a wave reach the same hub and exchanges on its list
// head would serialise.  Grid-stride over the vertices (whole waves, so the
// wave operations see every lane), a few workgroups per CU, each ending with
// one device-scope release.
template <class OffT>
__global__ __launch_bounds__(kBlock) void k_gh_sample(int64_t n, const OffT *__restrict__ off,
                                                      const int32_t *__restrict__ cols, int K,
                                                      const uint8_t *__restrict__ vmask, int32_t *cc,
                                                      int32_t *tu, int32_t *tv, int32_t *head,
                                                      int32_t *next,
                                                      const uint8_t *__restrict__ gsel) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = (int)(threadIdx.x & (kWave - 1));
  for (int64_t vw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; vw < n; vw += stride) {
    const int64_t v = vw + lane;
    // (in a batch hooked graph by graph, only the global sweep's graphs)
    const bool live = v < n && !(vmask && vmask[v]) && !(gsel && !gsel[v]);
    OffT b = 0;
    uint64_t deg = 0;
    if (live) {
      b = off[v];
      deg = (uint64_t)(off[v + 1] - b);
    }
    for (int r = 0; r < K; ++r) {
      int32_t x = -1, w = -1;
      if ((uint64_t)r < deg) {
        const uint64_t pos = deg <= (uint64_t)K ? (uint64_t)r
                                                : gh_mix(((uint64_t)v << 3) | (uint64_t)r) % deg;
        w = cols[b + (OffT)pos];
        if (w != (int32_t)v) x = hook_record<true>((int32_t)v, w, cc, tu, tv);
      }
      if (!head) continue;
      // arcs 2x = v->w (front of v's own list) and 2x+1 = w->v (front of w's)
      int2 nx = make_int2(-1, -1);
      if (x >= 0) nx.x = atomicExch(&head[v], 2 * x);
      nx.y = wave_push_front<4>(x >= 0, w, 2 * x + 1, head);
      if (x >= 0) reinterpret_cast<int2 *>(next)[x] = nx;
    }
  }
  block_release_device();
}

// One workgroup: roots of kGhSampleThreads * kGhSamplePer sampled vertices
// counted in LDS; the most frequent becomes the dominant root when it holds at
// least half of the (unmasked) samples, else -1.
__global__ __launch_bounds__(kGhSampleThreads) void k_gh_giant(int64_t n, const int32_t *__restrict__ cc,
                                                               const uint8_t *__restrict__ vmask,
                                                               int32_t *counters) {
  __shared__ int32_t keys[kGhHash];
  __shared__ int32_t cnts[kGhHash];
  __shared__ int s_valid;
  __shared__ unsigned long long s_best;
  const int t = threadIdx.x;
  for (int i = t; i < kGhHash; i += kGhSampleThreads) { keys[i] = -1; cnts[i] = 0; }
  if (t == 0) { s_valid = 0; s_best = 0ull; }
  __syncthreads();
  int valid = 0;
#pragma unroll
  for (int s = 0; s < kGhSamplePer; ++s) {
    const uint64_t i = (uint64_t)t * kGhSamplePer + s;
    const int32_t v = (int32_t)(gh_mix(0x5eedull ^ (i << 20)) % (uint64_t)n);
    if (vmask && vmask[v]) continue;
    ++valid;
    const int32_t r = gh_root(v, cc);
    uint32_t h = ((uint32_t)r * 0x9E3779B1u) >> (32 - 13);
    while (true) {   // at most 4096 keys in 8192 slots: a free slot exists
      const int32_t old = atomicCAS(&keys[h], -1, r);
      if (old == -1 || old == r) { atomicAdd(&cnts[h], 1); break; }
      h = (h + 1) & (kGhHash - 1);
    }
  }
  atomicAdd(&s_valid, valid);
  __syncthreads();
  for (int i = t; i < kGhHash; i += kGhSampleThreads)
    if (cnts[i] > 0)
      atomicMax(&s_best, ((unsigned long long)(uint32_t)cnts[i] << 32) | (uint32_t)keys[i]);
  __syncthreads();
  if (t == 0) {
    const int best = (int)(s_best >> 32);
    counters[kCntGiant] = (s_valid > 0 && 2 * best >= s_valid) ? (int32_t)(uint32_t)s_best : -1;
  }
}

// Batches: one workgroup per packed graph g finds the most frequent root among
// up to kGhBatchSamples of its (unmasked) vertices (all of them when it has no
// more) and writes it to giants[g] when it holds at least half of them, else
// -1; counters[kCntGiant] becomes 0 when some graph has one.  Skipping one
// dominant tree per graph is sound because no edge joins two packed graphs.
constexpr int kGhBatchThreads = 256;
constexpr int kGhBatchSamples = 1024;
constexpr int kGhBatchHash = 2048;
__global__ __launch_bounds__(kGhBatchThreads) void k_gh_giants(const int64_t *__restrict__ vtx_off,
                                                               const int32_t *__restrict__ cc,
                                                               const uint8_t *__restrict__ vmask,
                                                               const uint8_t *__restrict__ gsel,
                                                               int32_t *giants, int32_t *counters) {
  __shared__ int32_t keys[kGhBatchHash];
  __shared__ int32_t cnts[kGhBatchHash];
  __shared__ int s_valid;
  __shared__ unsigned long long s_best;
  const int t = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t lo = vtx_off[g], ng = vtx_off[g + 1] - lo;
  for (int i = t; i < kGhBatchHash; i += kGhBatchThreads) { keys[i] = -1; cnts[i] = 0; }
  if (t == 0) { s_valid = 0; s_best = 0ull; }
  __syncthreads();
  int valid = 0;
  for (int i = t; i < kGhBatchSamples && (int64_t)i < ng; i += kGhBatchThreads) {
    const int64_t off = ng <= kGhBatchSamples ? (int64_t)i
                                              : (int64_t)(gh_mix(((uint64_t)g << 20) ^ (uint64_t)i) % (uint64_t)ng);
    const int32_t v = (int32_t)(lo + off);
    if ((vmask && vmask[v]) || (gsel && !gsel[v])) continue;
    ++valid;
    const int32_t r = gh_root(v, cc);
    uint32_t h = ((uint32_t)r * 0x9E3779B1u) >> (32 - 11);
    while (true) {   // at most 1024 keys in 2048 slots: a free slot exists
      const int32_t old = atomicCAS(&keys[h], -1, r);
      if (old == -1 || old == r) { atomicAdd(&cnts[h], 1); break; }
      h = (h + 1) & (kGhBatchHash - 1);
    }
  }
  atomicAdd(&s_valid, valid);
  __syncthreads();
  for (int i = t; i < kGhBatchHash; i += kGhBatchThreads)
    if (cnts[i] > 0)
      atomicMax(&s_best, ((unsigned long long)(uint32_t)cnts[i] << 32) | (uint32_t)keys[i]);
  __syncthreads();
  if (t == 0) {
    const int best = (int)(s_best >> 32);
    const bool found = s_valid > 0 && 2 * best >= s_valid;
    store_agent(&giants[g], found ? (int32_t)(uint32_t)s_best : -1);
    if (found) atomicMax(&counters[kCntGiant], 0);
  }
}

// graph of vertex v: the last g with vtx_off[g] <= v
__device__ __forceinline__ int gh_graph_of(const int64_t *__restrict__ vtx_off, int G, int64_t v) {
  int lo = 0, hi = G;   // vtx_off[lo] <= v < vtx_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (vtx_off[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// The full sweep: a workgroup takes kGhThreads consecutive vertices at a
// time (grid-stride over such chunks, a few workgroups per CU), scans their
// degrees in LDS and walks the union of their arcs with unit stride (arcs
// already sampled are visited again and join nothing new).  With a dominant root D (counters
// [kCntGiant] >= 0; in a batch, giants[g] of the vertex's graph g) a vertex
// whose root is D offers nothing and the others offer every remaining arc;
// without one, an arc is hooked from its larger end only.  The arcs a wave keeps are queued in its own LDS region and hooked
// 64 at a time, so that every lane of a hooking wave carries a hook (without
// the queue half the lanes of a chain's waves idle through every hook).  Also
// counts the vertices whose first arc stays in their 8192-id
// tile (counters[kCntLocal]), so that a later call on the same buffers can
// tell whether the ids have gained locality.  Each workgroup ends with one
// device-scope release.
template <class OffT>
__global__ __launch_bounds__(kGhThreads, 8) void k_gh_sweep(int64_t n, const OffT *__restrict__ off,
                                                            const int32_t *__restrict__ cols,
                                                            const uint8_t *__restrict__ vmask,
                                                            int32_t *cc, int32_t *tu, int32_t *tv,
                                                            int32_t *head, int32_t *next,
                                                            int32_t *counters,
                                                            const int64_t *__restrict__ vtx_off,
                                                            int num_graphs,
                                                            const int32_t *__restrict__ giants,
                                                            const uint8_t *__restrict__ gsel,
                                                            int minhook) {
  __shared__ int s_scan[kGhThreads + 1];
  __shared__ OffT s_beg[kGhThreads];
  __shared__ int32_t s_min[kGhThreads];   // the first pass's edge (v, s_min) or -1
  __shared__ int s_wave[kGhThreads / kWave];
  __shared__ int2 s_q[kGhThreads / kWave][2 * kWave];   // per-wave queue of kept arcs
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  int2 *q = s_q[t / kWave];
  int qn = 0;   // queued arcs of this wave (the same in all its lanes)
  const int32_t giant = counters[kCntGiant];
  const int64_t chunks = (n + kGhThreads - 1) / kGhThreads;
  int locals = 0;
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int64_t v0 = c * kGhThreads;
    const int64_t v = v0 + t;
    int deg = 0;
    OffT beg = 0;
    // slot v holds (v, m) only when the first pass hooked v (a root never
    // records an edge that starts at itself before the sweep below); its
    // arcs go onto the lists here
    const int32_t mv = (minhook && v < n && tu[v] == (int32_t)v) ? tv[v] : -1;
    s_min[t] = mv;
    if (head && minhook) {
      // arc 2v = v -> mv onto v's own list, 2v+1 = mv -> v onto mv's, grouped
      // per wave by target (on graphs with hubs most vertices pick a hub)
      int2 nx = make_int2(-1, -1);
      if (mv >= 0) nx.x = atomicExch(&head[v], (int32_t)(2 * v));
      nx.y = wave_push_front<2>(mv >= 0, mv, (int32_t)(2 * v + 1), head);
      if (mv >= 0) reinterpret_cast<int2 *>(next)[v] = nx;
    }
    if (v < n && !(vmask && vmask[v]) && !(gsel && !gsel[v])) {
      const OffT b = off[v], e = off[v + 1];
      if (e > b) locals += (cols[b] >> kGhTileShift) == (int32_t)(v >> kGhTileShift);
      beg = b;
      if (e > beg) {
        // the dominant root this vertex's tree is compared with
        const int32_t d = giant < 0 ? -1
                        : giants ? giants[gh_graph_of(vtx_off, num_graphs, v)] : giant;
        if (!(d >= 0 && find_root((int32_t)v, cc) == d)) deg = (int)(e - beg);
      }
    }
    s_beg[t] = beg;
    int total;
    const int excl = block_excl_scan<kGhThreads>(deg, s_wave, &total);
    s_scan[t] = excl;
    if (t == kGhThreads - 1) s_scan[kGhThreads] = excl + deg;
    __syncthreads();
    for (int b0 = 0; b0 < total; b0 += kGhThreads) {
      const int k = b0 + t;
      bool keep = false;
      int32_t u = 0, w = 0;
      if (k < total) {
        const int j = lds_upper_search(s_scan, kGhThreads, k);
        u = (int32_t)(v0 + j);
        w = cols[s_beg[j] + (OffT)(k - s_scan[j])];
        keep = (giant >= 0 ? w != u : w < u) && w != s_min[j];
      }
      const uint64_t m = __ballot(keep);
      if (keep) q[qn + lanes_below(m)] = make_int2(u, w);
      qn += (int)__popcll(m);
      if (qn >= kWave) {
        // the wave's own LDS writes above are read back by other lanes
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const int2 e = q[lane];
        const int2 rest = q[kWave + lane];
        qn -= kWave;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (lane < qn) q[lane] = rest;
        hook_edge<true>(e.x, e.y, cc, tu, tv, head, next);
      }
    }
    __syncthreads();   // s_scan and s_beg are rewritten for the next chunk
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  if (lane < qn) {
    const int2 e = q[lane];
    hook_edge<true>(e.x, e.y, cc, tu, tv, head, next);
  }
  for (int o = 32; o > 0; o >>= 1) locals += __shfl_xor(locals, o, 64);
  if ((t & 63) == 0 && locals) atomicAdd(&counters[kCntLocal], locals);
  block_release_device();
}

// One workgroup: the share of sampled arcs that leave their source's 8192-id
// tile (counters[kCntProbeArcs], counters[kCntProbeCross]); up to 4 arcs of
// each of kGhSampleThreads * kGhSamplePer sampled vertices.
template <class OffT>
__global__ __launch_bounds__(kGhSampleThreads) void k_gh_probe(int64_t n, const OffT *__restrict__ off,
                                                               const int32_t *__restrict__ cols,
                                                               const uint8_t *__restrict__ vmask,
                                                               int32_t *counters) {
  int arcs = 0, cross = 0;
#pragma unroll
  for (int s = 0; s < kGhSamplePer; ++s) {
    const uint64_t i = (uint64_t)threadIdx.x * kGhSamplePer + s;
    const int64_t v = (int64_t)(gh_mix(0x9b0beull ^ (i << 20)) % (uint64_t)n);
    if (vmask && vmask[v]) continue;
    const OffT b = off[v], e = off[v + 1];
    for (OffT a = b; a < e && a < b + 4; ++a) {
      ++arcs;
      cross += (cols[a] >> kGhTileShift) != (int32_t)(v >> kGhTileShift);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    arcs += __shfl_xor(arcs, o, 64);
    cross += __shfl_xor(cross, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&counters[kCntProbeArcs], arcs);
    atomicAdd(&counters[kCntProbeCross], cross);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Grid of the hooking kernels: every workgroup ends with a device-scope
// release (a write-back of its XCD's L2), so they loop over their work with
// `per_cu` workgroups per CU instead of one workgroup per piece.
static unsigned gh_grid(const rst_ctx *ctx, unsigned pieces, int per_cu) {
  const unsigned cap = (unsigned)(ctx->num_cus * per_cu);
  return pieces < cap ? pieces : cap;
}

int ghook_sample_arcs(const rst_ctx *ctx, const rst_csr *g) {
  if (ctx->opt.hook_sample >= 0) return ctx->opt.hook_sample;
  // sampling pays where the average degree is well above a chain's or a mesh's
  return g->nnz >= 6 * g->n ? 2 : 0;
}

rst_status enqueue_hook_global(rst_ctx *ctx, const rst_csr *g, ForestBufs &f, bool init) {
  const int64_t n = g->n;
  const int K = ghook_sample_arcs(ctx, g);
  // the first pass needs every vertex a root with an empty slot (fresh init);
  // it serves sweeps without a dominant tree (on graphs with random ids and
  // hubs it leaves many small trees where sampling finds the dominant one:
  // C3's sweep 0.05 -> 1.7 ms with it in place of the sampled hooks)
  const int minhook = (init && K == 0 && !f.gsel) ? 1 : 0;
  RST_KMARK(ctx, RST_KERNEL_HOOK_SAMPLE, 0);
  if (init) {
    RST_SWEEP(ctx, k_gh_init, n, n, f.cc, f.tu, f.tv, f.head);
    RST_HIP(hipGetLastError());
  }
  if (minhook) {
    if (g->offset_bytes == 4)
      hipLaunchKernelGGL(k_gh_minhook<int32_t>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0,
                         ctx->stream, n, (const int32_t *)g->offsets, g->cols, f.vmask, f.cc,
                         f.tu, f.tv);
    else
      hipLaunchKernelGGL(k_gh_minhook<int64_t>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0,
                         ctx->stream, n, (const int64_t *)g->offsets, g->cols, f.vmask, f.cc,
                         f.tu, f.tv);
    RST_HIP(hipGetLastError());
  }
  if (K > 0) {
    const unsigned sgrid = gh_grid(ctx, grid_for(n, kBlock), 8);
    if (g->offset_bytes == 4)
      hipLaunchKernelGGL(k_gh_sample<int32_t>, dim3(sgrid), dim3(kBlock), 0, ctx->stream, n,
                         (const int32_t *)g->offsets, g->cols, K, f.vmask, f.cc, f.tu, f.tv,
                         f.head, f.next, f.gsel);
    else
      hipLaunchKernelGGL(k_gh_sample<int64_t>, dim3(sgrid), dim3(kBlock), 0, ctx->stream, n,
                         (const int64_t *)g->offsets, g->cols, K, f.vmask, f.cc, f.tu, f.tv,
                         f.head, f.next, f.gsel);
    RST_HIP(hipGetLastError());
    if (f.giants && f.num_graphs > 1) {
      RST_TRY(enqueue_fill(ctx, f.counters + kCntGiant, 1, -1));
      hipLaunchKernelGGL(k_gh_giants, dim3(f.num_graphs), dim3(kGhBatchThreads), 0, ctx->stream,
                         f.vtx_off, f.cc, f.vmask, f.gsel, f.giants, f.counters);
    } else {
      hipLaunchKernelGGL(k_gh_giant, dim3(1), dim3(kGhSampleThreads), 0, ctx->stream, n, f.cc,
                         f.vmask, f.counters);
    }
    RST_HIP(hipGetLastError());
  } else {
    RST_TRY(enqueue_fill(ctx, f.counters + kCntGiant, 1, -1));
  }
  RST_KMARK(ctx, RST_KERNEL_HOOK_SAMPLE, 1);
  RST_KMARK(ctx, RST_KERNEL_HOOK_GLOBAL, 0);
  const unsigned grid = gh_grid(ctx, grid_for(n, kGhThreads), 2);
  // per-graph dominant roots only when they were sought (sampling ran)
  const int32_t *batch_giants = (K > 0 && f.giants && f.num_graphs > 1) ? f.giants : nullptr;
  if (g->offset_bytes == 4)
    hipLaunchKernelGGL(k_gh_sweep<int32_t>, dim3(grid), dim3(kGhThreads), 0, ctx->stream, n,
                       (const int32_t *)g->offsets, g->cols, f.vmask, f.cc, f.tu, f.tv, f.head,
                       f.next, f.counters, f.vtx_off, f.num_graphs, batch_giants, f.gsel, minhook);
  else
    hipLaunchKernelGGL(k_gh_sweep<int64_t>, dim3(grid), dim3(kGhThreads), 0, ctx->stream, n,
                       (const int64_t *)g->offsets, g->cols, f.vmask, f.cc, f.tu, f.tv, f.head,
                       f.next, f.counters, f.vtx_off, f.num_graphs, batch_giants, f.gsel, minhook);
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_HOOK_GLOBAL, 1);
  return RST_OK;
}

rst_status enqueue_locality_probe(rst_ctx *ctx, const rst_csr *g, const uint8_t *vmask,
                                  int32_t *counters) {
  if (g->offset_bytes == 4)
    hipLaunchKernelGGL(k_gh_probe<int32_t>, dim3(1), dim3(kGhSampleThreads), 0, ctx->stream, g->n,
                       (const int32_t *)g->offsets, g->cols, vmask, counters);
  else
    hipLaunchKernelGGL(k_gh_probe<int64_t>, dim3(1), dim3(kGhSampleThreads), 0, ctx->stream, g->n,
                       (const int64_t *)g->offsets, g->cols, vmask, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

}  // namespace rst
