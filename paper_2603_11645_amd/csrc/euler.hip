// euler.hip -- Euler-tour rooting of a spanning forest (Sec. III-D).
//
// Arc numbering: the forest edge held by slot x gives twin arcs 2x = (tu->tv)
// and 2x+1 = (tv->tu), so rev(e) = e ^ 1 and no compaction pass is needed (a
// slot whose vertex stayed a component root is empty).  The paper sorts the
// arcs only to make every vertex's out-arcs form one list; any cyclic order of
// them yields a valid tour, so the per-vertex lists are built here by linking
// each arc in front of its source's list with one atomic exchange
// (head[v], next[e]).
//
// Successor (the equation of Sec. III-D): succ(e) = next(rev e) if that is not
// -1, else the first arc of from(rev e) = to(e).  Cycle breaking: the arc whose
// successor would wrap around to the root's first out-arc is the reverse of
// the root's last out-arc, i.e. an arc e into a root with next(rev e) = -1;
// it gets succ -1.  Both rules are applied in one pass that also initialises
// the ranking words.
//
// List ranking (Wyllie pointer jumping): each arc holds a packed 64-bit word
// (succ in the low half, hops-to-succ in the high half); a round replaces it by
// (succ of succ, own hops + hops of succ).  The word is read and written with
// single 64-bit accesses, so every read sees a consistent pair and rounds can
// update in place: a read of an already-advanced neighbour only moves the
// reader further.  After ceil(log2 L) rounds every word holds (-1, distance to
// the tail of its list).
//
// Parent rule: of the twins e=(u->v) and rev e, the one with the larger
// distance to the tail comes first in the tour; it is the downward traversal,
// so P[v] = u.  Component roots get P[r] = r.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

__device__ __forceinline__ uint64_t pack_rank(int32_t succ, uint32_t hops) {
  return ((uint64_t)hops << 32) | (uint32_t)succ;
}

__device__ __forceinline__ bool is_root(int32_t v, const int32_t *cc, const int32_t *comp_root) {
  const int32_t c = cc[v];
  const int32_t d = comp_root[c];
  return d == v || (d == -1 && c == v);
}

// Designated roots: claim their component, P[r] = r.
__global__ void k_mark_roots(const int32_t *__restrict__ roots, int32_t nroots, int64_t n,
                             const int32_t *__restrict__ cc, int32_t *comp_root, int32_t *parent,
                             int32_t *counters) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nroots) return;
  const int32_t r = roots[i];
  if (r < 0 || r >= n) {
    atomicOr(&counters[kCntRangeErr], 1);
    return;
  }
  const int32_t old = atomicCAS(&comp_root[cc[r]], -1, r);
  if (old != -1 && old != r) atomicOr(&counters[kCntRootErr], 1);
  parent[r] = r;
}

// Per-vertex out-arc lists: next[e] = previous head of src(e), head = e.
template <int B>
__global__ __launch_bounds__(B) void k_link(int64_t slots, const int32_t *__restrict__ tu,
                                                 const int32_t *__restrict__ tv, int32_t *head,
                                                 int32_t *next) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= slots) return;
  const int32_t a = tu[x];
  int2 nx = make_int2(-1, -1);
  if (a >= 0) {
    const int32_t b = tv[x];
    nx.x = atomicExch(&head[a], (int32_t)(2 * x));
    nx.y = atomicExch(&head[b], (int32_t)(2 * x + 1));
  }
  reinterpret_cast<int2 *>(next)[x] = nx;
}

// Successor + cycle break + rank init for both arcs of a slot.
__global__ __launch_bounds__(kBlock) void k_succ(int64_t slots, const int32_t *__restrict__ tu,
                                                 const int32_t *__restrict__ tv,
                                                 const int32_t *__restrict__ head,
                                                 const int32_t *__restrict__ next,
                                                 const int32_t *__restrict__ cc,
                                                 const int32_t *__restrict__ comp_root,
                                                 uint64_t *rank) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= slots) return;
  const int32_t a = tu[x];
  ulonglong2 out;
  if (a < 0) {
    out.x = pack_rank(-1, 0);
    out.y = pack_rank(-1, 0);
  } else {
    const int32_t b = tv[x];
    const int2 nx = reinterpret_cast<const int2 *>(next)[x];
    // arc 2x = a->b, its reverse is 2x+1 = b->a
    int32_t s0 = nx.y;
    if (s0 == -1) s0 = is_root(b, cc, comp_root) ? -1 : head[b];
    int32_t s1 = nx.x;
    if (s1 == -1) s1 = is_root(a, cc, comp_root) ? -1 : head[a];
    out.x = pack_rank(s0, s0 >= 0 ? 1u : 0u);
    out.y = pack_rank(s1, s1 >= 0 ? 1u : 0u);
  }
  reinterpret_cast<ulonglong2 *>(rank)[x] = out;
}

__global__ __launch_bounds__(kBlock) void k_rank_init(int64_t A, const int32_t *__restrict__ succ,
                                                      uint64_t *rank) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A) return;
  int32_t s = succ[e];
  if (s < 0 || s >= A) s = -1;   // out-of-range successors end the list (no wild gathers)
  rank[e] = pack_rank(s, s >= 0 ? 1u : 0u);
}

// One pointer-jumping round over A words, EPT words per thread; all gathers of
// a thread are issued before any of them is consumed.
template <int EPT>
__global__ __launch_bounds__(kBlock) void k_rank_round(int64_t A, uint64_t *rank) {
  const int64_t base = (int64_t)blockIdx.x * (kBlock * EPT) + threadIdx.x;
  uint64_t me[EPT], nb[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int64_t i = base + (int64_t)j * kBlock;
    me[j] = i < A ? rank[i] : pack_rank(-1, 0);
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int32_t s = (int32_t)(uint32_t)me[j];
    nb[j] = s >= 0 ? rank[s] : 0ull;
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int32_t s = (int32_t)(uint32_t)me[j];
    if (s >= 0) {
      const uint64_t hops = (me[j] >> 32) + (nb[j] >> 32);
      rank[base + (int64_t)j * kBlock] = (hops << 32) | (nb[j] & 0xffffffffull);
    }
  }
}

// ---------------------------------------------------------------------------
// Tiled list ranking.  Arcs are cut into tiles of kRankTile consecutive ids.
// Inside a tile the list splits into segments (maximal runs whose successor
// stays in the tile); a workgroup ranks its tile's segments by pointer jumping
// in LDS, so each arc learns the last arc of its segment (its "exit") and the
// hops to it.  Only the exits -- arcs whose successor leaves the tile, and
// list tails -- form the contracted list, which is ranked by Wyllie rounds;
// a final pass adds each arc's in-tile hops to its exit's contracted distance.
// When arc ids follow the tour's geometry (tiles of the hooking stage line up
// with tiles of arcs) almost every successor stays in its tile and the global
// pointer-jumping traffic shrinks by orders of magnitude; without locality the
// contracted list is about as long as the input and the cost is that of plain
// Wyllie plus two streaming passes.
//
// Word encoding after the tile pass: a non-exit arc e holds (exit of e, hops
// to it), whose first half lies in e's own tile; an exit keeps (successor, 1)
// with the successor outside the tile, or (-1, 0) at a list tail.
// ---------------------------------------------------------------------------
constexpr int kRankTile = 16384;
constexpr int kRankThreads = 1024;
constexpr int kRankPer = kRankTile / kRankThreads;
constexpr int kRuler = 8;                            // every 8th arc is a ruler
constexpr int kStrided = kRankTile / kRuler;         // 2048 strided ruler slots
constexpr int kRulerSlots = 3584;                    // + up to 1536 extra segment heads

__device__ __forceinline__ bool in_tile(int32_t id, int64_t e) {
  return id >= 0 && ((int64_t)id / kRankTile) == (e / kRankTile);
}

// endsucc[v]: successor of an arc into v whose reverse ends v's out-arc list,
// i.e. the first out-arc of v, or -1 (cycle break) when v is its tree's root.
template <int B>
__global__ __launch_bounds__(B) void k_endsucc(int64_t n, const int32_t *__restrict__ head,
                                                    const int32_t *__restrict__ cc,
                                                    const int32_t *__restrict__ comp_root,
                                                    int32_t *endsucc) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) endsucc[v] = is_root((int32_t)v, cc, comp_root) ? -1 : head[v];
}

struct SlotSrc {            // arcs described by the forest slots (fused successor pass)
  const int32_t *tu, *tv, *next, *endsucc;
};

// Within a tile: every segment head and every 8th arc is a ruler.  Each ruler
// walks its piece of list (to the next ruler or the segment's exit) in LDS;
// the rulers are then ranked by pointer jumping, and a second walk writes
// (exit, hops to exit) for every arc.  Total LDS work is two linear passes;
// each thread walks two rulers at once so their LDS latencies overlap.  A
// tile with more segment heads than ruler slots (no locality) is ranked by
// plain pointer jumping in LDS instead.
template <bool kFromSlots>
__global__ __launch_bounds__(kRankThreads) void k_rank_tile(int64_t A, uint64_t *rank, int32_t *xid,
                                                            int32_t *exits, int32_t *tile_exits,
                                                            SlotSrc src) {
  __shared__ int16_t ls[kRankTile];                  // local successor, -1 at an exit
  __shared__ __align__(16) unsigned char region[kRankTile * 2];   // flags+rulers, or hop counts
  __shared__ int s_extra;
  __shared__ int s_nexit;
  uint32_t *haspred = reinterpret_cast<uint32_t *>(region);          // [kRankTile / 32] bits
  int16_t *r_start = reinterpret_cast<int16_t *>(region + kRankTile / 8);
  int16_t *r_next = r_start + kRulerSlots;
  uint16_t *r_len = reinterpret_cast<uint16_t *>(r_next + kRulerSlots);
  int16_t *r_exit = reinterpret_cast<int16_t *>(r_len + kRulerSlots);
  uint16_t *dd = reinterpret_cast<uint16_t *>(region);             // fallback: [kRankTile]

  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * kRankTile;
  const int cnt = (int)((A - e0) < kRankTile ? (A - e0) : kRankTile);
  if (tid == 0) { s_extra = 0; s_nexit = 0; }
  for (int q = tid; q < kRankTile / 32; q += kRankThreads) haspred[q] = 0u;
  __syncthreads();
  // two half-passes of 8 arcs per thread: loads of a half are issued together
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    constexpr int H = kRankPer / 2;
    uint64_t w[H];
    if (kFromSlots) {
      // successor: next(rev e), or at the end of dst's list endsucc[dst]
      int32_t dst[H], sc[H];
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int64_t e = e0 + tid + (h * H + j) * kRankThreads;
        dst[j] = -1; sc[j] = -1;
        if (e < A) {
          const int32_t a = src.tu[e >> 1];
          dst[j] = a < 0 ? -1 : ((e & 1) ? a : src.tv[e >> 1]);   // 2x = a->b, 2x+1 = b->a
          sc[j] = src.next[e ^ 1];
        }
      }
#pragma unroll
      for (int j = 0; j < H; ++j)
        if (dst[j] >= 0 && sc[j] == -1) sc[j] = src.endsucc[dst[j]];
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int32_t t = dst[j] < 0 ? -1 : sc[j];
        w[j] = pack_rank(t, t >= 0 ? 1u : 0u);
      }
    } else {
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int i = tid + (h * H + j) * kRankThreads;
        w[j] = i < cnt ? rank[e0 + i] : 0ull;
      }
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int i = tid + (h * H + j) * kRankThreads;
      bool is_exit = false;
      if (i < cnt) {
        const int32_t sc = (int32_t)(uint32_t)w[j];
        const int64_t sl = (int64_t)sc - e0;
        if (sc >= 0 && sl >= 0 && sl < cnt) {
          ls[i] = (int16_t)sl;
          atomicOr(&haspred[sl >> 5], 1u << (sl & 31));
        } else {
          ls[i] = -1;
          is_exit = true;
        }
      }
      // exits of tile b go to exits[b*kRankTile + k], k from an LDS counter
      const int slot = wave_append(is_exit, &s_nexit);
      if (is_exit) {
        exits[e0 + slot] = (int32_t)(e0 + i);
        if (kFromSlots) rank[e0 + i] = w[j];
      }
      if (i < cnt) xid[e0 + i] = is_exit ? slot : 0;
    }
  }
  __syncthreads();
  // strided rulers own slots 0..kStrided-1; heads off the stride get extra slots
  for (int q = tid; q < kStrided; q += kRankThreads) r_start[q] = (int16_t)(q * kRuler);
#pragma unroll
  for (int j = 0; j < kRankPer; ++j) {
    const int i = tid + j * kRankThreads;
    if (i < cnt && (i % kRuler) != 0 && !((haspred[i >> 5] >> (i & 31)) & 1u)) {
      const int x = atomicAdd(&s_extra, 1);
      if (kStrided + x < kRulerSlots) r_start[kStrided + x] = (int16_t)i;
    }
  }
  __syncthreads();
  if (tid == 0) tile_exits[blockIdx.x] = s_nexit;
  const int extra = s_extra;
  if (kStrided + extra <= kRulerSlots) {
    const int nslots = kStrided + extra;
    // walk 1, two rulers per thread in lock step: hops to the next ruler or exit
    for (int qb = tid; qb < nslots; qb += 2 * kRankThreads) {
      int q[2] = {qb, qb + kRankThreads};
      int jj[2], len[2] = {0, 0}, nx[2] = {-1, -1}, ex[2] = {0, 0};
      bool act[2];
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        jj[w] = q[w] < nslots ? r_start[q[w]] : cnt;
        act[w] = jj[w] < cnt;
      }
      while (act[0] || act[1]) {
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          if (!act[w]) continue;
          const int sj = ls[jj[w]];
          if (sj < 0) { ex[w] = jj[w]; act[w] = false; continue; }
          jj[w] = sj;
          ++len[w];
          if ((sj % kRuler) == 0) { nx[w] = sj / kRuler; act[w] = false; continue; }
          if (len[w] > cnt) { ex[w] = sj; act[w] = false; }   // only on a cycle
        }
      }
#pragma unroll
      for (int w = 0; w < 2; ++w)
        if (q[w] < nslots) {
          r_next[q[w]] = (int16_t)nx[w];
          r_len[q[w]] = (uint16_t)len[w];
          r_exit[q[w]] = (int16_t)ex[w];
        }
    }
    __syncthreads();
    // pointer jumping over the rulers
    constexpr int QP = (kRulerSlots + kRankThreads - 1) / kRankThreads;
    for (int round = 0; round < 13; ++round) {
      int16_t nn[QP], ne[QP];
      uint16_t nl[QP];
      bool changed = false;
#pragma unroll
      for (int k = 0; k < QP; ++k) {
        const int q = tid + k * kRankThreads;
        if (q < nslots) {
          const int x = r_next[q];
          nn[k] = (int16_t)x; nl[k] = r_len[q]; ne[k] = r_exit[q];
          if (x >= 0) {
            nn[k] = r_next[x];
            nl[k] = (uint16_t)(r_len[q] + r_len[x]);
            ne[k] = r_exit[x];
            changed = true;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < QP; ++k) {
        const int q = tid + k * kRankThreads;
        if (q < nslots) { r_next[q] = nn[k]; r_len[q] = nl[k]; r_exit[q] = ne[k]; }
      }
      if (!__syncthreads_or(changed)) break;
    }
    // walk 2: every non-exit arc gets (exit, hops to exit).  The rulers' data
    // go to registers first; then the region holds per-arc hop counts and ls
    // the local exit of each arc it is done with, so that the rank words are
    // written once, coalesced, at the end (written along the list they
    // landed in partial lines).
    int w_st[QP], w_tot[QP], w_ex[QP];
#pragma unroll
    for (int k = 0; k < QP; ++k) {
      const int q = tid + k * kRankThreads;
      w_st[k] = q < nslots ? r_start[q] : cnt;
      w_tot[k] = q < nslots ? r_len[q] : 0;
      w_ex[k] = q < nslots ? r_exit[q] : 0;
    }
    __syncthreads();
    uint16_t *hp = reinterpret_cast<uint16_t *>(region);     // [kRankTile] hops to exit
#pragma unroll
    for (int k = 0; k < QP; k += 2) {
      int jj[2], k2[2] = {0, 0};
      bool act[2];
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        jj[w] = (k + w < QP) ? w_st[k + w] : cnt;
        act[w] = jj[w] < cnt;
      }
      while (act[0] || act[1]) {
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          if (!act[w]) continue;
          const int sj = ls[jj[w]];
          if (sj < 0 || k2[w] > cnt) { act[w] = false; continue; }
          hp[jj[w]] = (uint16_t)(w_tot[k + w] - k2[w]);
          ls[jj[w]] = (int16_t)w_ex[k + w];
          jj[w] = sj;
          ++k2[w];
          if ((sj % kRuler) == 0) act[w] = false;
        }
      }
    }
    __syncthreads();
    // exits keep the word of the first pass; every other arc now has its exit
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
      const int i = tid + j * kRankThreads;
      if (i < cnt && ls[i] >= 0) rank[e0 + i] = pack_rank((int32_t)(e0 + ls[i]), hp[i]);
    }
    return;
  }
  // fallback: pointer jumping over all arcs of the tile (ls as pointers, dd as hops)
#pragma unroll
  for (int j = 0; j < kRankPer; ++j) {
    const int i = tid + j * kRankThreads;
    if (i < cnt) {
      const int sj = ls[i];
      dd[i] = sj < 0 ? 0 : 1;
      ls[i] = (int16_t)(sj < 0 ? i : sj);
    }
  }
  __syncthreads();
  for (int round = 0; round < 15; ++round) {
    int16_t np[kRankPer];
    uint16_t nd[kRankPer];
    bool changed = false;
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
      const int i = tid + j * kRankThreads;
      if (i < cnt) {
        const int q = ls[i];
        np[j] = ls[q];
        nd[j] = (uint16_t)(dd[i] + dd[q]);
        changed |= (np[j] != q);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
      const int i = tid + j * kRankThreads;
      if (i < cnt) { ls[i] = np[j]; dd[i] = nd[j]; }
    }
    if (!__syncthreads_or(changed)) break;
  }
#pragma unroll
  for (int j = 0; j < kRankPer; ++j) {
    const int i = tid + j * kRankThreads;
    if (i < cnt && ls[i] != i) rank[e0 + i] = pack_rank((int32_t)(e0 + ls[i]), dd[i]);
  }
}

// Exclusive scan of the per-tile exit counts (one block): base[b], base[tiles] = M.
__global__ __launch_bounds__(1024) void k_tile_scan(const int32_t *__restrict__ cnt, int64_t tiles,
                                                    int64_t *base) {
  __shared__ int s_wave[1024 / kWave];
  __shared__ int64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < tiles; b0 += 1024) {
    const int64_t b = b0 + threadIdx.x;
    const int x = b < tiles ? cnt[b] : 0;
    int total;
    const int excl = block_excl_scan<1024>(x, s_wave, &total);
    if (b < tiles) base[b] = s_carry + excl;
    __syncthreads();
    if (threadIdx.x == 0) s_carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) base[tiles] = s_carry;
}

__device__ __forceinline__ int64_t exit_index(int32_t ex, const int32_t *xid, const int64_t *base) {
  return base[ex / kRankTile] + xid[ex];
}

// Contracted list over the exits (one block per tile): next exit and weighted
// hops to it.
__global__ __launch_bounds__(kBlock) void k_rank_contract(const int32_t *__restrict__ exits,
                                                          const int32_t *__restrict__ tile_exits,
                                                          const int64_t *__restrict__ base,
                                                          const uint64_t *__restrict__ rank,
                                                          const int32_t *__restrict__ xid,
                                                          uint64_t *crank) {
  const int64_t e0 = (int64_t)blockIdx.x * kRankTile;
  const int cntb = tile_exits[blockIdx.x];
  const int64_t b0 = base[blockIdx.x];
  for (int j = threadIdx.x; j < cntb; j += kBlock) {
    const int32_t x = exits[e0 + j];
    const int32_t s = (int32_t)(uint32_t)rank[x];
    if (s < 0) {
      crank[b0 + j] = pack_rank(-1, 0);
      continue;
    }
    const uint64_t ws = rank[s];
    const int32_t id = (int32_t)(uint32_t)ws;
    int32_t ex = s;
    uint32_t dl = 0;
    if (in_tile(id, s)) { ex = id; dl = (uint32_t)(ws >> 32); }
    crank[b0 + j] = pack_rank((int32_t)exit_index(ex, xid, base), 1u + dl);
  }
}

// The contracted list (M = base[tiles] words) ranked by one block: pointer
// jumping in LDS until no word has a successor left, so the round count needs
// no host round trip.  Longer lists (more than kSmallLds words; one CU would
// be slower on them than multi-block rounds) raise counters[kCntRankOverflow]
// and change nothing: the consumers then skip their work and the host ranks
// the list in multi-block rounds.  counters[kCntExits] = M, counters[kCntRankRounds] =
// rounds.
constexpr int kSmallThreads = 1024;
constexpr int kSmallPer = 19;
// 19456 words of 8 B (152 KB; the block-wide OR reduction takes a little LDS too)
constexpr int kSmallLds = kSmallPer * kSmallThreads;

__global__ __launch_bounds__(kSmallThreads) void k_rank_small(const int64_t *__restrict__ Mp,
                                                              uint64_t *crank, int32_t *counters) {
  __shared__ uint64_t s_word[kSmallLds];   // (succ, hops) as in crank
  const int tid = threadIdx.x;
  const int64_t M = *Mp;
  if (tid == 0) counters[kCntExits] = (int32_t)M;
  int rounds = 0;
  // a list of M words needs at most ceil(log2 M) rounds; the cap also ends the
  // loop on malformed (cyclic) input
  int max_rounds = 1;
  while (((int64_t)1 << max_rounds) < M) ++max_rounds;
  if (M <= kSmallLds) {
    // Each thread keeps its own words in registers; a round gathers the
    // successors' words from LDS, then (after a barrier) publishes its own.
    const int m = (int)M;
    uint64_t own[kSmallPer];
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const int i = tid + k * kSmallThreads;
      own[k] = i < m ? crank[i] : pack_rank(-1, 0);
      if (i < m) s_word[i] = own[k];
    }
    bool active = __syncthreads_or(1);
    while (active) {
      bool more = false;
#pragma unroll
      for (int k = 0; k < kSmallPer; ++k) {
        const int32_t sc = (int32_t)(uint32_t)own[k];
        if (sc >= 0) {
          const uint64_t nb = s_word[sc];
          own[k] = (((own[k] >> 32) + (nb >> 32)) << 32) | (nb & 0xffffffffull);
          more |= (int32_t)(uint32_t)nb >= 0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kSmallPer; ++k) {
        const int i = tid + k * kSmallThreads;
        if (i < m) s_word[i] = own[k];
      }
      ++rounds;
      active = __syncthreads_or(more) && rounds < max_rounds;
    }
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const int i = tid + k * kSmallThreads;
      if (i < m) crank[i] = own[k];
    }
  } else {
    if (tid == 0) counters[kCntRankOverflow] = 1;
    return;
  }
  if (tid == 0) counters[kCntRankRounds] = rounds;
}

// dist[e] = hops to its exit + contracted distance of that exit, stored as (-1, dist)
__global__ __launch_bounds__(kBlock) void k_rank_expand(int64_t A, uint64_t *rank,
                                                        const int32_t *__restrict__ xid,
                                                        const int64_t *__restrict__ base,
                                                        const uint64_t *__restrict__ crank,
                                                        const int32_t *__restrict__ counters) {
  if (counters[kCntRankOverflow]) return;   // contracted list not ranked yet
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A) return;
  const uint64_t w = rank[e];
  const int32_t id = (int32_t)(uint32_t)w;
  uint32_t dist;
  if (in_tile(id, e))
    dist = (uint32_t)(w >> 32) + (uint32_t)(crank[exit_index(id, xid, base)] >> 32);
  else
    dist = (uint32_t)(crank[exit_index((int32_t)e, xid, base)] >> 32);
  rank[e] = pack_rank(-1, dist);
}

__device__ __forceinline__ uint32_t arc_dist(int64_t e, const uint64_t *__restrict__ rank,
                                             const int32_t *__restrict__ xid,
                                             const int64_t *__restrict__ base,
                                             const uint64_t *__restrict__ crank) {
  const uint64_t w = rank[e];
  const int32_t id = (int32_t)(uint32_t)w;
  if (in_tile(id, e)) return (uint32_t)(w >> 32) + (uint32_t)(crank[exit_index(id, xid, base)] >> 32);
  return (uint32_t)(crank[exit_index((int32_t)e, xid, base)] >> 32);
}

// Distances of both arcs of a slot, then the parent rule; default component
// roots get P[v] = v and are counted.
template <int B>
__global__ __launch_bounds__(B) void k_expand_parent(int64_t slots, int64_t n,
                                                          const int32_t *__restrict__ tu,
                                                          const int32_t *__restrict__ tv,
                                                          const uint64_t *__restrict__ rank,
                                                          const int32_t *__restrict__ xid,
                                                          const int64_t *__restrict__ base,
                                                          const uint64_t *__restrict__ crank,
                                                          const int32_t *__restrict__ cc,
                                                          const int32_t *__restrict__ comp_root,
                                                          int32_t *parent, int32_t *counters) {
  if (counters[kCntRankOverflow]) return;   // contracted list not ranked yet (block-uniform)
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < slots) {
    const int32_t a = tu[x];
    if (a >= 0) {
      const int32_t b = tv[x];
      const uint32_t d0 = arc_dist(2 * x, rank, xid, base, crank);
      const uint32_t d1 = arc_dist(2 * x + 1, rank, xid, base, crank);
      if (d0 > d1) parent[b] = a;   // a->b comes first in the tour: it descends
      else parent[a] = b;
    }
  }
  bool comp = false;
  if (x < n) {
    comp = cc[x] == (int32_t)x;
    if (comp && comp_root[x] == -1) parent[x] = (int32_t)x;
  }
  wave_count(comp, &counters[kCntComponents]);
}

__global__ __launch_bounds__(kBlock) void k_rank_extract(int64_t A, const uint64_t *__restrict__ rank,
                                                         int32_t *dist) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < A) dist[e] = (int32_t)(rank[e] >> 32);
}

// Parents from tour order (slots) + default component roots (vertices).
__global__ __launch_bounds__(kBlock) void k_parent(int64_t slots, int64_t n,
                                                   const int32_t *__restrict__ tu,
                                                   const int32_t *__restrict__ tv,
                                                   const uint64_t *__restrict__ rank,
                                                   const int32_t *__restrict__ cc,
                                                   const int32_t *__restrict__ comp_root,
                                                   int32_t *parent, int32_t *counters) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < slots) {
    const int32_t a = tu[x];
    if (a >= 0) {
      const int32_t b = tv[x];
      const ulonglong2 r = reinterpret_cast<const ulonglong2 *>(rank)[x];
      const uint32_t d0 = (uint32_t)(r.x >> 32), d1 = (uint32_t)(r.y >> 32);
      if (d0 > d1) parent[b] = a;   // a->b comes first: it descends
      else parent[a] = b;           // b->a comes first: b is a's parent
    }
  }
  bool comp = false;
  if (x < n) {
    comp = cc[x] == (int32_t)x;
    if (comp && comp_root[x] == -1) parent[x] = (int32_t)x;
  }
  wave_count(comp, &counters[kCntComponents]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int rank_rounds_for(int64_t max_list_len) {
  int r = 0;
  while (((int64_t)1 << r) < max_list_len) ++r;
  return r;
}

rst_status enqueue_mark_roots(rst_ctx *ctx, const int32_t *roots, int32_t nroots, int64_t n,
                              const int32_t *cc, int32_t *comp_root, int32_t *parent,
                              int32_t *counters) {
  if (nroots <= 0) return RST_OK;
  hipLaunchKernelGGL(k_mark_roots, dim3(grid_for(nroots, kBlock)), dim3(kBlock), 0, ctx->stream,
                     roots, nroots, n, cc, comp_root, parent, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_link(rst_ctx *ctx, int64_t slots, const int32_t *tu, const int32_t *tv,
                        int32_t *head, int32_t *next) {
  if (slots <= 0) return RST_OK;
  RST_KMARK(ctx, RST_KERNEL_LINK, 0);
  RST_SWEEP(ctx, k_link, slots, slots, tu, tv, head, next);
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_LINK, 1);
  return RST_OK;
}

rst_status enqueue_succ(rst_ctx *ctx, int64_t slots, const int32_t *tu, const int32_t *tv,
                        const int32_t *head, const int32_t *next, const int32_t *cc,
                        const int32_t *comp_root, uint64_t *rank) {
  if (slots <= 0) return RST_OK;
  hipLaunchKernelGGL(k_succ, dim3(grid_for(slots, kBlock)), dim3(kBlock), 0, ctx->stream, slots,
                     tu, tv, head, next, cc, comp_root, rank);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_rank_init(rst_ctx *ctx, int64_t A, const int32_t *succ, uint64_t *rank) {
  if (A <= 0) return RST_OK;
  hipLaunchKernelGGL(k_rank_init, dim3(grid_for(A, kBlock)), dim3(kBlock), 0, ctx->stream, A,
                     succ, rank);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

template <int EPT>
static rst_status launch_rounds(rst_ctx *ctx, int64_t A, uint64_t *rank, int rounds) {
  const unsigned grid = grid_for(A, kBlock * EPT);
  for (int r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(k_rank_round<EPT>, dim3(grid), dim3(kBlock), 0, ctx->stream, A, rank);
    RST_HIP(hipGetLastError());
  }
  return RST_OK;
}

rst_status enqueue_rank_rounds(rst_ctx *ctx, int64_t A, uint64_t *rank, int rounds,
                               hipEvent_t ev_begin, hipEvent_t ev_end) {
  if (ev_begin) RST_HIP(hipEventRecord(ev_begin, ctx->stream));
  if (A > 0 && rounds > 0) {
    switch (ctx->opt.rank_elems_per_thread) {
      case 1: RST_TRY(launch_rounds<1>(ctx, A, rank, rounds)); break;
      case 2: RST_TRY(launch_rounds<2>(ctx, A, rank, rounds)); break;
      case 8: RST_TRY(launch_rounds<8>(ctx, A, rank, rounds)); break;
      default: RST_TRY(launch_rounds<4>(ctx, A, rank, rounds)); break;
    }
  }
  if (ev_end) RST_HIP(hipEventRecord(ev_end, ctx->stream));
  return RST_OK;
}

size_t rank_exit_capacity(int64_t A) { return (size_t)(A + 1); }
size_t rank_tile_count(int64_t A) { return (size_t)((A + kRankTile - 1) / kRankTile); }

rst_status enqueue_rank_tiled(rst_ctx *ctx, int64_t A, uint64_t *rank, int32_t *xid,
                              const RankBufs &rb, int32_t *counters, const SlotArcs *from_slots,
                              bool expand) {
  if (A <= 0) return RST_OK;
  const int64_t tiles = (int64_t)rank_tile_count(A);
  if (from_slots) {
    RST_SWEEP(ctx, k_endsucc, from_slots->n, from_slots->n, from_slots->head, from_slots->cc,
              from_slots->comp_root, from_slots->endsucc);
    RST_HIP(hipGetLastError());
    SlotSrc src{from_slots->tu, from_slots->tv, from_slots->next, from_slots->endsucc};
    RST_KMARK(ctx, RST_KERNEL_RANK_TILE, 0);
    hipLaunchKernelGGL(k_rank_tile<true>, dim3((unsigned)tiles), dim3(kRankThreads), 0, ctx->stream,
                       A, rank, xid, rb.exits, rb.tile_exits, src);
  } else {
    SlotSrc src{};
    RST_KMARK(ctx, RST_KERNEL_RANK_TILE, 0);
    hipLaunchKernelGGL(k_rank_tile<false>, dim3((unsigned)tiles), dim3(kRankThreads), 0,
                       ctx->stream, A, rank, xid, rb.exits, rb.tile_exits, src);
  }
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_RANK_TILE, 1);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, ctx->stream, rb.tile_exits, tiles,
                     rb.tile_base);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_rank_contract, dim3((unsigned)tiles), dim3(kBlock), 0, ctx->stream, rb.exits,
                     rb.tile_exits, rb.tile_base, rank, xid, rb.crank);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_rank_small, dim3(1), dim3(kSmallThreads), 0, ctx->stream,
                     rb.tile_base + tiles, rb.crank, counters);
  RST_HIP(hipGetLastError());
  if (expand) RST_TRY(enqueue_rank_expand(ctx, A, rank, xid, rb, counters));
  return RST_OK;
}

rst_status enqueue_rank_expand(rst_ctx *ctx, int64_t A, uint64_t *rank, const int32_t *xid,
                               const RankBufs &rb, const int32_t *counters) {
  hipLaunchKernelGGL(k_rank_expand, dim3(grid_for(A, kBlock)), dim3(kBlock), 0, ctx->stream, A,
                     rank, xid, rb.tile_base, rb.crank, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status rank_overflow_fallback(rst_ctx *ctx, const RankBufs &rb, int32_t *counters) {
  int64_t M = ctx->host_pinned[kCntExits];
  if (M < 0) return RST_E_DEVICE;
  const int rounds = rank_rounds_for(M);
  RST_TRY(enqueue_rank_rounds(ctx, M, rb.crank, rounds, nullptr, nullptr));
  RST_TRY(enqueue_fill(ctx, counters + kCntRankOverflow, 1, 0));
  RST_TRY(enqueue_fill(ctx, counters + kCntRankRounds, 1, rounds));
  return RST_OK;
}

rst_status enqueue_expand_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                                 const int32_t *tv, const uint64_t *rank, const int32_t *xid,
                                 const int64_t *tile_base, const uint64_t *crank, const int32_t *cc,
                                 const int32_t *comp_root, int32_t *parent, int32_t *counters) {
  const int64_t items = slots > n ? slots : n;
  RST_SWEEP(ctx, k_expand_parent, items, slots, n, tu, tv, rank, xid, tile_base, crank, cc,
            comp_root, parent, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_rank_extract(rst_ctx *ctx, int64_t A, const uint64_t *rank, int32_t *dist) {
  if (A <= 0) return RST_OK;
  hipLaunchKernelGGL(k_rank_extract, dim3(grid_for(A, kBlock)), dim3(kBlock), 0, ctx->stream, A,
                     rank, dist);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                          const int32_t *tv, const uint64_t *rank, const int32_t *cc,
                          const int32_t *comp_root, int32_t *parent, int32_t *counters) {
  const int64_t items = slots > n ? slots : n;
  hipLaunchKernelGGL(k_parent, dim3(grid_for(items, kBlock)), dim3(kBlock), 0, ctx->stream, slots,
                     n, tu, tv, rank, cc, comp_root, parent, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

}  // namespace rst
