// unionfind.h -- union-find steps in global memory shared by the hooking
// kernels (hook.hip, ghook.hip): root finding with path halving, the Euler arc
// pair of a recorded edge, and the hook of Sec. III-B with its edge recorded
// at the hooked root (Sec. I).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace rst {

// Root of x with path halving.  Invariant cc[y] <= y (equality iff y is a root)
// makes the walk strictly decreasing, so it ends even on stale reads; the
// stores (agent scope, see store_agent) only ever replace a non-root's pointer
// by one of its ancestors.
__device__ __forceinline__ int32_t find_root(int32_t x, int32_t *cc) {
  int32_t cur = cc[x];
  if (cur != x) {
    int32_t prev = x, nxt;
    while (cur > (nxt = cc[cur])) {
      store_agent(&cc[prev], nxt);
      prev = cur;
      cur = nxt;
    }
  }
  return cur;
}

// Arcs 2x = a->b and 2x+1 = b->a of the edge recorded at slot x, each put in
// front of its source's list.
__device__ __forceinline__ void link_slot(int32_t x, int32_t a, int32_t b, int32_t *head,
                                          int32_t *next) {
  int2 nx;
  nx.x = atomicExch(&head[a], 2 * x);
  nx.y = atomicExch(&head[b], 2 * x + 1);
  reinterpret_cast<int2 *>(next)[x] = nx;
}

// Hook the trees of u and v; on success record (u,v) at the hooked root (and
// link its two arcs when head is non-NULL).
template <bool kRecord>
__device__ __forceinline__ void hook_edge(int32_t u, int32_t v, int32_t *cc, int32_t *tu,
                                          int32_t *tv, int32_t *head = nullptr,
                                          int32_t *next = nullptr) {
  int32_t ru = find_root(u, cc);
  int32_t rv = find_root(v, cc);
  while (ru != rv) {
    const int32_t lo = ru < rv ? ru : rv;
    const int32_t hi = ru < rv ? rv : ru;
    const int32_t old = atomicCAS(&cc[hi], hi, lo);
    if (old == hi) {
      if (kRecord) {
        tu[hi] = u;
        tv[hi] = v;
        if (head) link_slot(hi, u, v, head, next);
      }
      return;
    }
    // hi was hooked meanwhile: continue from its new parent (an ancestor)
    if (ru == hi) ru = old; else rv = old;
  }
}

}  // namespace rst
