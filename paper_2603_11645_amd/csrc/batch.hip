// batch.hip -- many graphs packed into one CSR (global vertex ids) processed in
// one pass.  Graphs never share a component, so the forest stages run over the
// packed graph unchanged: cycle breaking happens once per designated root, the
// generalisation to forests of Sec. III-D.  The number of launches does not
// depend on the number of graphs: per-graph work is expressed as per-vertex
// masks and per-root seeds, built here with one block per graph.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

// vmask[v] = method of v's graph (nonzero: not hooked, handled by BFS)
__global__ __launch_bounds__(kBlock) void k_graph_mask(const int64_t *__restrict__ vtx_off,
                                                       const uint8_t *__restrict__ method,
                                                       uint8_t *vmask) {
  const int g = blockIdx.x;
  const int64_t b = vtx_off[g], e = vtx_off[g + 1];
  const uint8_t m = method[g];
  for (int64_t v = b + threadIdx.x; v < e; v += kBlock) vmask[v] = m;
}

// Hooking variant per graph of a batch (GConn+Euler graphs; BFS graphs get 0):
// up to 4 arcs of each of up to kSplitSamples pseudo-randomly chosen vertices,
// and the share of them that leave their source's 8192-id tile.  More than
// half: the graph's ids carry no locality and the global sweep hooks it
// (gsel 1 for its vertices), else the tile pass (gsel 0).
constexpr int kSplitThreads = 256;
constexpr int kSplitSamples = 1024;
constexpr int kSplitTileShift = 13;   // the tile pass's 8192-id tiles

__device__ __forceinline__ uint64_t split_mix(uint64_t z) {   // splitmix64 finaliser
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <class OffT>
__global__ __launch_bounds__(kSplitThreads) void k_batch_hook_split(const int64_t *__restrict__ vtx_off,
                                                                    const OffT *__restrict__ off,
                                                                    const int32_t *__restrict__ cols,
                                                                    const uint8_t *__restrict__ method,
                                                                    uint8_t *gsel) {
  __shared__ int s_arcs, s_cross;
  const int g = blockIdx.x;
  const int64_t lo = vtx_off[g], ng = vtx_off[g + 1] - lo;
  if (threadIdx.x == 0) { s_arcs = 0; s_cross = 0; }
  __syncthreads();
  if (!method[g]) {
    int arcs = 0, cross = 0;
    for (int i = threadIdx.x; i < kSplitSamples && (int64_t)i < ng; i += kSplitThreads) {
      const int64_t v = lo + (ng <= kSplitSamples ? (int64_t)i
                                                  : (int64_t)(split_mix(((uint64_t)g << 20) ^ i) %
                                                              (uint64_t)ng));
      const OffT b = off[v], e = off[v + 1];
      for (OffT a = b; a < e && a < b + 4; ++a) {
        ++arcs;
        cross += (cols[a] >> kSplitTileShift) != (int32_t)(v >> kSplitTileShift);
      }
    }
    atomicAdd(&s_arcs, arcs);
    atomicAdd(&s_cross, cross);
  }
  __syncthreads();
  const uint8_t sel = (!method[g] && 2 * s_cross > s_arcs) ? 1 : 0;
  for (int64_t v = lo + threadIdx.x; v < lo + ng; v += kSplitThreads) gsel[v] = sel;
}

// Consistency of the offset tables and roots: vtx_off non-decreasing, the
// arc table matching the CSR offsets, every root inside its own graph.
template <class OffT>
__global__ __launch_bounds__(kBlock) void k_batch_check(int32_t G, int64_t n, int64_t nnz,
                                                        const OffT *__restrict__ off,
                                                        const int64_t *__restrict__ vtx_off,
                                                        const int64_t *__restrict__ arc_off,
                                                        const int32_t *__restrict__ roots,
                                                        int32_t *counters) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int64_t b = vtx_off[g], e = vtx_off[g + 1];
  bool bad = b < 0 || e < b || e > n || (g == 0 && b != 0) || (g == G - 1 && e != n);
  if (!bad) {
    bad = arc_off[g] != (int64_t)off[b] || arc_off[g + 1] != (int64_t)off[e] ||
          (g == G - 1 && arc_off[g + 1] != nnz);
    const int32_t r = roots[g];
    bad = bad || r < b || r >= e;
  }
  if (bad) atomicOr(&counters[kCntRangeErr], 1);
}

// Validation of a batch's arcs: every neighbour id of graph g lies in
// [vtx_off[g], vtx_off[g+1]) (the graph of an arc is found by binary search
// in arc_off); otherwise graphs would share components.
__global__ __launch_bounds__(kBlock) void k_batch_arcs_check(int32_t G, int64_t nnz,
                                                             const int64_t *__restrict__ vtx_off,
                                                             const int64_t *__restrict__ arc_off,
                                                             const int32_t *__restrict__ cols,
                                                             int32_t *counters) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nnz) return;
  int lo = 0, hi = G;   // largest g in [0, G) with arc_off[g] <= a
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (arc_off[mid] <= a) lo = mid; else hi = mid;
  }
  const int32_t c = cols[a];
  if (c < vtx_off[lo] || c >= vtx_off[lo + 1]) atomicOr(&counters[kCntBatchArcErr], 1);
}

rst_status enqueue_batch_arcs_check(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                    int32_t *counters) {
  if (g->nnz <= 0) return RST_OK;
  hipLaunchKernelGGL(k_batch_arcs_check, dim3(grid_for(g->nnz, kBlock)), dim3(kBlock), 0,
                     ctx->stream, b->num_graphs, g->nnz, b->vtx_off, b->arc_off, g->cols, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

// counters[kCntBatchBfs] = graphs with a nonzero method (BFS),
// counters[kCntBatchBfsVtx] = their vertices
__global__ __launch_bounds__(kBlock) void k_count_methods(int32_t G,
                                                          const int64_t *__restrict__ vtx_off,
                                                          const uint8_t *__restrict__ m,
                                                          int32_t *counters) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const bool bfs = g < G && m[g] != 0;
  wave_count(bfs, &counters[kCntBatchBfs]);
  if (bfs) atomicAdd(&counters[kCntBatchBfsVtx], (int32_t)(vtx_off[g + 1] - vtx_off[g]));
}

__global__ void k_copy_u8(const uint8_t *__restrict__ src, uint8_t *dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i] ? 1 : 0;
}

__global__ void k_fill_u8(uint8_t *dst, int64_t count, uint8_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = value;
}

// The offset tables of a batch holding one graph (all n vertices, root r).
__global__ void k_single_batch(int64_t n, int64_t nnz, int32_t root, int64_t *vtx_off,
                               int64_t *arc_off, int32_t *roots) {
  if (threadIdx.x == 0) {
    vtx_off[0] = 0; vtx_off[1] = n;
    arc_off[0] = 0; arc_off[1] = nnz;
    roots[0] = root;
  }
}

rst_status enqueue_single_batch(rst_ctx *ctx, const rst_csr *g, int32_t root, int64_t *vtx_off,
                                int64_t *arc_off, int32_t *roots) {
  hipLaunchKernelGGL(k_single_batch, dim3(1), dim3(64), 0, ctx->stream, g->n, g->nnz, root, vtx_off,
                     arc_off, roots);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_graph_mask(rst_ctx *ctx, const rst_batch *b, const uint8_t *method,
                              uint8_t *vmask) {
  hipLaunchKernelGGL(k_graph_mask, dim3((unsigned)b->num_graphs), dim3(kBlock), 0, ctx->stream,
                     b->vtx_off, method, vmask);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_batch_hook_split(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                    const uint8_t *method, uint8_t *gsel) {
  if (g->offset_bytes == 4)
    hipLaunchKernelGGL(k_batch_hook_split<int32_t>, dim3((unsigned)b->num_graphs),
                       dim3(kSplitThreads), 0, ctx->stream, b->vtx_off,
                       (const int32_t *)g->offsets, g->cols, method, gsel);
  else
    hipLaunchKernelGGL(k_batch_hook_split<int64_t>, dim3((unsigned)b->num_graphs),
                       dim3(kSplitThreads), 0, ctx->stream, b->vtx_off,
                       (const int64_t *)g->offsets, g->cols, method, gsel);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_batch_check(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                               int32_t *counters) {
  const unsigned grid = grid_for(b->num_graphs, kBlock);
  if (g->offset_bytes == 4)
    hipLaunchKernelGGL(k_batch_check<int32_t>, dim3(grid), dim3(kBlock), 0, ctx->stream,
                       b->num_graphs, g->n, g->nnz, (const int32_t *)g->offsets, b->vtx_off,
                       b->arc_off, b->roots, counters);
  else
    hipLaunchKernelGGL(k_batch_check<int64_t>, dim3(grid), dim3(kBlock), 0, ctx->stream,
                       b->num_graphs, g->n, g->nnz, (const int64_t *)g->offsets, b->vtx_off,
                       b->arc_off, b->roots, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_count_methods(rst_ctx *ctx, const rst_batch *b, const uint8_t *m,
                                 int32_t *counters) {
  const int32_t G = b->num_graphs;
  hipLaunchKernelGGL(k_count_methods, dim3(grid_for(G, kBlock)), dim3(kBlock), 0, ctx->stream, G,
                     b->vtx_off, m, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_copy_u8(rst_ctx *ctx, const uint8_t *src, uint8_t *dst, int64_t count) {
  if (count <= 0) return RST_OK;
  hipLaunchKernelGGL(k_copy_u8, dim3(grid_for(count, kBlock)), dim3(kBlock), 0, ctx->stream, src,
                     dst, count);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_fill_u8(rst_ctx *ctx, uint8_t *dst, int64_t count, uint8_t value) {
  if (count <= 0) return RST_OK;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(count, kBlock)), dim3(kBlock), 0, ctx->stream, dst,
                     count, value);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

}  // namespace rst
