// device_common.h -- wavefront/block primitives for gfx950 (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rst {

// number of set bits of `mask` below this lane (mbcnt over the 64-bit mask)
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// inclusive prefix sum across the 64 lanes of a wave
__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive prefix sum over a block of BLOCK threads.  s_wave needs BLOCK/64
// ints of LDS.  Returns the exclusive prefix; *total gets the block sum.  Ends
// with a barrier so s_wave can be reused.
template <int BLOCK>
__device__ __forceinline__ int block_excl_scan(int x, int *s_wave, int *total) {
  const int incl = wave_incl_scan(x);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) s_wave[wid] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) {
    const int s = s_wave[w];
    off += (w < wid) ? s : 0;
    tot += s;
  }
  *total = tot;
  __syncthreads();
  return incl - x + off;
}

// Append the lanes with `pred` set to a global queue: one atomic per wave.
// Must be called by all lanes of the wave (uniform control flow).  Returns the
// slot of this lane (valid only where pred is true).
__device__ __forceinline__ int wave_append(bool pred, int32_t *counter) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return -1;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  int base = 0;
  if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(counter, (int)__popcll(mask));
  base = __shfl(base, leader, 64);
  return base + lanes_below(mask);
}

// Sum of `x` over the wave, added once per wave to *counter.
__device__ __forceinline__ void wave_count(bool pred, int32_t *counter) {
  const uint64_t mask = __ballot(pred);
  if (mask && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)mask) - 1)
    atomicAdd(counter, (int)__popcll(mask));
}

// largest j in [0, len) with s[j] <= k, given s[0] <= k < s[len] (LDS array)
__device__ __forceinline__ int lds_upper_search(const int *s, int len, int k) {
  int lo = 0, hi = len;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s[mid] <= k) lo = mid; else hi = mid;
  }
  return lo;
}

// Store at agent scope (global_store with the sc1 bit on gfx950).  Used for
// every write of a union-find label or an arc-list head made while hooking is
// in progress or before it: kernels on other XCDs later compare-and-swap,
// exchange, overwrite or read these words.  With plain stores, a path-halving
// store left in one XCD's L2 was seen to land in memory after the final
// pointer-jumping pass had written the same word from another XCD (a label
// one hop short of the root, a few vertices in 1 of 40 calls; measured on
// MI355X), which a release fence at the end of each wave did not prevent.
__device__ __forceinline__ void store_agent(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-scope release by the calling wave (agent-scope fence: this XCD's L2
// is written back).  Kernels whose waves hook trees through compare-and-swap
// and path-halving stores in global memory, from many workgroups at once, end
// every wave with it: without it, a hook made by such a kernel was now and
// then not yet seen by the kernels after it on other XCDs (measured on
// MI355X).
__device__ __forceinline__ void wave_release_device() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

// The same for a whole workgroup at once (called by all its threads): each
// wave waits until its own stores and atomics have completed, the barrier
// orders them before one wave's release fence, and that fence (which writes
// back this XCD's L2 as a whole) releases them all.  One write-back per
// workgroup instead of one per wave: when every wave of a large grid fenced,
// the write-backs queued up (measured on MI355X).
__device__ __forceinline__ void block_release_device() {
  __builtin_amdgcn_s_waitcnt(0);   // vmcnt, expcnt and lgkmcnt all zero
  __syncthreads();
  if (threadIdx.x < 64) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

}  // namespace rst
