// verify.hip -- device check that a parent array is a rooted spanning forest
// of the graph under the library's root convention (the problem statement of
// Sec. I, applied per component: the component of `root` is rooted at root,
// every other component at its minimum vertex id).  Used by the autotuner to
// reject any candidate setting whose output is wrong, and exported as
// rst_verify.
//
// A parent array passes when (1) every entry is a vertex id, (2) exactly the
// designated roots are their own parents, (3) every other vertex's parent is
// one of its neighbours, and (4) following parents from any vertex reaches a
// designated root of the same component (checked by ceil(log2 n) + 1 rounds
// of pointer jumping, so a cycle anywhere leaves some vertex on a non-root).
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

enum { kVerBad = 0, kVerFirst = 1 };

__device__ __forceinline__ void ver_fail(int64_t v, int32_t *vc) {
  atomicAdd(&vc[kVerBad], 1);
  atomicMin(&vc[kVerFirst], (int32_t)v);
}

template <class OffT>
__global__ __launch_bounds__(kBlock) void k_verify_local(int64_t n, const OffT *__restrict__ off,
                                                         const int32_t *__restrict__ cols,
                                                         const int32_t *__restrict__ label,
                                                         int32_t root,
                                                         const int32_t *__restrict__ parent,
                                                         int32_t *anc, int32_t *vc) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t p = parent[v];
  const int32_t lv = label[v];
  const bool designated = v == root || (lv == (int32_t)v && lv != label[root]);
  bool bad = p < 0 || p >= n;
  if (!bad) {
    if (designated) {
      bad = p != (int32_t)v;
    } else if (p == (int32_t)v) {
      bad = true;
    } else {
      bool found = false;
      for (int64_t a = (int64_t)off[v]; a < (int64_t)off[v + 1] && !found; ++a)
        found = cols[a] == p;
      bad = !found;
    }
  }
  anc[v] = bad ? (int32_t)v : p;
  if (bad) ver_fail(v, vc);
}

__global__ __launch_bounds__(kBlock) void k_verify_jump(int64_t n, const int32_t *__restrict__ a,
                                                        int32_t *b) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) b[v] = a[a[v]];
}

__global__ __launch_bounds__(kBlock) void k_verify_reach(int64_t n, const int32_t *__restrict__ anc,
                                                         const int32_t *__restrict__ parent,
                                                         const int32_t *__restrict__ label,
                                                         int32_t *vc) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t x = anc[v];
  if (parent[x] != x || label[x] != label[v]) ver_fail(v, vc);
}

rst_status enqueue_verify(rst_ctx *ctx, const rst_csr *g, int32_t root, const int32_t *label,
                          const int32_t *parent, int32_t *anc0, int32_t *anc1, int32_t *vc) {
  const int64_t n = g->n;
  const unsigned grid = grid_for(n, kBlock);
  if (g->offset_bytes == 4)
    hipLaunchKernelGGL(k_verify_local<int32_t>, dim3(grid), dim3(kBlock), 0, ctx->stream, n,
                       (const int32_t *)g->offsets, g->cols, label, root, parent, anc0, vc);
  else
    hipLaunchKernelGGL(k_verify_local<int64_t>, dim3(grid), dim3(kBlock), 0, ctx->stream, n,
                       (const int64_t *)g->offsets, g->cols, label, root, parent, anc0, vc);
  RST_HIP(hipGetLastError());
  int rounds = 1;
  while (((int64_t)1 << rounds) < n) ++rounds;
  ++rounds;
  int32_t *a = anc0, *b = anc1;
  for (int r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(k_verify_jump, dim3(grid), dim3(kBlock), 0, ctx->stream, n, a, b);
    RST_HIP(hipGetLastError());
    int32_t *t = a; a = b; b = t;
  }
  hipLaunchKernelGGL(k_verify_reach, dim3(grid), dim3(kBlock), 0, ctx->stream, n, a, parent, label,
                     vc);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

}  // namespace rst
