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

// Hook the trees of u and v by compare-and-swap of the larger root; on
// success record (u,v) at the hooked root and return that root (the slot),
// else -1 (u and v were already in one tree).  kTestFirst: read the root's
// word before the compare-and-swap and skip it when the root has been hooked
// already (the word of a hooked root only ever moves up its ancestors, so
// the value read is a valid next step).  Where many lanes reach the same few
// roots at once (sampled arcs into hubs) the failing compare-and-swaps on one
// address serialised: testing first cut the sampling pass of an R-MAT graph
// with hubs of degree 1.6e5 from 1.17 to 0.68 ms; where almost every
// compare-and-swap succeeds (a chain's sweep) the extra load cost 3%.
template <bool kTestFirst = false>
__device__ __forceinline__ int32_t hook_record(int32_t u, int32_t v, int32_t *cc, int32_t *tu,
                                               int32_t *tv) {
  int32_t ru = find_root(u, cc);
  int32_t rv = find_root(v, cc);
  while (ru != rv) {
    const int32_t lo = ru < rv ? ru : rv;
    const int32_t hi = ru < rv ? rv : ru;
    int32_t old = hi;
    if (kTestFirst) old = cc[hi];
    if (old == hi) old = atomicCAS(&cc[hi], hi, lo);
    if (old == hi) {
      tu[hi] = u;
      tv[hi] = v;
      return hi;
    }
    // hi was hooked meanwhile: continue from its new parent (an ancestor)
    if (ru == hi) ru = old; else rv = old;
  }
  return -1;
}

// Join the trees of u and v, recording nothing (labels only); kTestFirst as
// for hook_record.
template <bool kTestFirst>
__device__ __forceinline__ void hook_join(int32_t u, int32_t v, int32_t *cc) {
  int32_t ru = find_root(u, cc);
  int32_t rv = find_root(v, cc);
  while (ru != rv) {
    const int32_t lo = ru < rv ? ru : rv;
    const int32_t hi = ru < rv ? rv : ru;
    int32_t old = hi;
    if (kTestFirst) old = cc[hi];
    if (old == hi) old = atomicCAS(&cc[hi], hi, lo);
    if (old == hi) return;
    if (ru == hi) ru = old; else rv = old;
  }
}

// Hook the trees of u and v; on success record (u,v) at the hooked root (and
// link its two arcs when head is non-NULL).
template <bool kRecord>
__device__ __forceinline__ void hook_edge(int32_t u, int32_t v, int32_t *cc, int32_t *tu,
                                          int32_t *tv, int32_t *head = nullptr,
                                          int32_t *next = nullptr) {
  if (kRecord) {
    const int32_t x = hook_record(u, v, cc, tu, tv);
    if (x >= 0 && head) link_slot(x, u, v, head, next);
    return;
  }
  hook_join<false>(u, v, cc);
}

// Put `item` in front of list `key` (head[key]) for every lane with `pred`,
// and return the item that follows it.  Called by all lanes of the wave.
// Lanes pushing onto the same list are chained among themselves in lane order
// and the chain is linked in with one exchange by its lowest lane: on graphs
// with hubs many lanes of a wave push onto one hub's list, and exchanges on
// one address serialise.  Groups are formed for up to kRounds keys (each time
// the key of the lowest lane not yet grouped); every other lane exchanges on
// its own, all exchanges issued together.
template <int kRounds>
__device__ __forceinline__ int32_t wave_push_front(bool pred, int32_t key, int32_t item,
                                                   int32_t *head) {
  const int lane = lane_id();
  uint64_t pend = __ballot(pred);
  int leader = lane;   // the lane that exchanges for this lane's group
  int nl = -1;         // the next lane of the group (-1: the group's last)
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (!pend) break;
    const int first = __ffsll((unsigned long long)pend) - 1;
    const int32_t k = __shfl(key, first, 64);
    const uint64_t grp = __ballot(pred && key == k) & pend;
    if ((grp >> lane) & 1ull) {
      leader = first;
      const uint64_t above = lane == 63 ? 0ull : grp & (~0ull << (lane + 1));
      nl = above ? __ffsll((unsigned long long)above) - 1 : -1;
    }
    pend &= ~grp;
  }
  const int32_t after = __shfl(item, nl >= 0 ? nl : lane, 64);
  int32_t old = -1;
  if (pred && leader == lane) old = atomicExch(&head[key], item);
  const int32_t tail_next = __shfl(old, leader, 64);
  return nl >= 0 ? after : tail_next;
}

}  // namespace rst
