// glrank.hip -- list ranking by a sparse ruling set in global memory
// (Sec. III-D "parallel list ranking"), for tours whose arc ids carry no
// locality: random vertex ids (R-MAT, permuted meshes, long chains), where
// the per-tile ranking of euler.hip finds almost every arc at a tile exit.
//
// Level 1 works on one int32 word per arc: first the successor (-1 at a list
// tail, -2 for an arc that belongs to no list), then, once a walk has passed
// it, the arc's code (ruler << 8 | offset).  Every arc with id = 0 mod k and
// every list head starts a ruler; one thread walks from each ruler along the
// list until the next ruler or the tail, overwriting each arc it passes with
// its code (the arc is read once, then written once, by that thread alone).
// A walk that reaches 255 arcs opens a new ruler (numbered after the others
// by an atomic counter) so offsets fit 8 bits.  Each ruler leaves one 64-bit
// word (next ruler or -1 : 32, hops to it : 32) -- a weighted list of about
// A/k words, ranked the same way at the next level (64-bit words, weighted
// offsets, a new ruler opened after kGlUpperCap words: a level's kernel takes
// as long as its longest piece, and above level 1 each walk has a whole
// thread to itself), until the list fits one workgroup, which ranks it in LDS
// by pointer jumping.  Each level's codes then become distances to the tail
// (ruler distance less the offset), from the top level down; the consumer of
// level 1 (the parent rule, or the plain distances) does the last expansion
// on the fly.
//
// Distances follow the words' meaning: (next, w) says dist(word) = w +
// dist(next), and (-1, w) says dist(word) = w.  A unit-weight arc has w = 1,
// a tail w = 0.
//
// Rulers chosen by id are spread like random samples on a list with random
// ids (pieces of mean length k) and exactly every k-th arc on a list with
// consecutive ids.  Ruler ids of level 1 must fit 24 bits; more than
// kGlHeadCap list heads or more rulers than that raise a flag and every
// kernel after the walks does nothing; the caller then ranks by Wyllie rounds.
#include "rst_internal.h"
#include "device_common.h"

namespace rst {

constexpr int kGlThreads = 256;
constexpr int kGlOffBits = 8;
constexpr int kGlCap = (1 << kGlOffBits) - 1;           // a walk opens a ruler after 255 arcs
constexpr int64_t kGlRidLimit = (int64_t)1 << (32 - kGlOffBits);   // level-1 ruler ids
constexpr int kGlFinalThreads = 1024;
constexpr int kGlFinalPer = 16;
constexpr int kGlFinal = kGlFinalThreads * kGlFinalPer;  // words ranked in LDS by one workgroup
constexpr int64_t kGlHeadCap = (int64_t)1 << 20;          // list heads (trees) handled
constexpr int kGlUpperCap = 63;                           // words per piece above level 1
constexpr uint64_t kGlHole = 0x00000000fffffffeull;       // (next -2, w 0): a word of no list

__device__ __forceinline__ uint64_t gl_pack(int32_t next, uint32_t w) {
  return ((uint64_t)w << 32) | (uint32_t)next;
}

// Words of level `level` (1 = the arcs): every level above the first holds
// the strided rulers, the heads and the opened rulers of the one below
// (dyn1: rulers opened at level 1; lvl[l]: at level l >= 2).
__device__ __forceinline__ int64_t gl_words(int level, int64_t A, int k1, int k, int64_t H,
                                            int64_t dyn1, const int32_t *lvl) {
  int64_t N = A;
  if (level >= 2) N = (A + k1 - 1) / k1 + H + dyn1;
  for (int l = 3; l <= level; ++l) N = (N + k - 1) / k + H + lvl[l - 1];
  return N;
}

// ---------------------------------------------------------------------------
// front ends: level-1 words and list heads
// ---------------------------------------------------------------------------

// Arcs from forest slots (the successor equation of Sec. III-D with the cycle
// break folded into endsucc): slot x = edge (a, b) gives arc 2x = a->b with
// successor next(2x+1), or endsucc[b] at the end of b's list, and arc 2x+1 =
// b->a likewise; an empty slot's arcs belong to no list.  A vertex v whose
// tree it roots (endsucc[v] = -1) and that has arcs contributes its first
// out-arc head[v] as a list head.
template <int B>
__global__ __launch_bounds__(B) void k_gslot_words(int64_t slots, int64_t n,
                                                   const int32_t *__restrict__ tu,
                                                   const int32_t *__restrict__ tv,
                                                   const int32_t *__restrict__ next,
                                                   const int32_t *__restrict__ endsucc,
                                                   const int32_t *__restrict__ head, int32_t *w1,
                                                   int32_t *heads, int64_t hcap, int32_t *counters) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < slots) {
    const int32_t a = tu[x];
    int2 out = make_int2(-2, -2);
    if (a >= 0) {
      const int32_t b = tv[x];
      const int2 nx = reinterpret_cast<const int2 *>(next)[x];
      out.x = nx.y != -1 ? nx.y : endsucc[b];
      out.y = nx.x != -1 ? nx.x : endsucc[a];
    }
    reinterpret_cast<int2 *>(w1)[x] = out;
  }
  bool is_head = false;
  int32_t h = -1;
  if (x < n && endsucc[x] == -1) {
    h = head[x];
    is_head = h >= 0;
  }
  const int slot = wave_append(is_head, &counters[kCntGHeads]);
  if (is_head && slot < hcap) heads[slot] = h;
}

// Arbitrary lists: level-1 words from succ (out-of-range successors end the
// list) and one has-predecessor byte per node.
__global__ __launch_bounds__(kGlThreads) void k_glist_words(int64_t A, const int32_t *__restrict__ succ,
                                                            int32_t *w1, uint8_t *haspred) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A) return;
  int32_t s = succ[e];
  if (s < -1 || s >= A) s = -1;
  w1[e] = s;
  if (s >= 0) haspred[s] = 1;
}

// Nodes without a predecessor are the list heads.
__global__ __launch_bounds__(kGlThreads) void k_glist_heads(int64_t A, const uint8_t *__restrict__ haspred,
                                                            int32_t *heads, int64_t hcap,
                                                            int32_t *counters) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool is_head = e < A && !haspred[e];
  const int slot = wave_append(is_head, &counters[kCntGHeads]);
  if (is_head && slot < hcap) heads[slot] = (int32_t)e;
}

// ---------------------------------------------------------------------------
// the walk of one level
// ---------------------------------------------------------------------------

// Ruler q < Rs starts at word q*k; ruler Rs + j at heads_in[j] (when that word
// is strided it is already ruler h/k: the head's slot is left a hole, and the
// head list of the next level names h/k); further rulers are opened by walks
// that reach the piece cap.  Each ruler's word of the next level goes to
// rw_out[ruler].
// kW01 (32-bit words only): the arcs weigh 1 when their id has an even number
// of one bits and 0 otherwise (the down and up arcs of a tour by parent
// edges, whose preorder count this ranks), instead of 1 each; a code's offset
// is then the weight walked since the ruler, still at most the piece's arcs.
template <bool kL1, bool kW01 = false>
__global__ __launch_bounds__(kGlThreads) void k_gwalk(int level, int64_t A, int k1, int k,
                                                      void *words, const int32_t *heads_in,
                                                      int32_t *heads_out, uint64_t *rw_out,
                                                      int64_t rw_cap, int64_t hcap,
                                                      int32_t *counters, int32_t *lvl) {
  if (counters[kCntGOverflow]) return;
  const int64_t H = counters[kCntGHeads];
  if (H > hcap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&counters[kCntGOverflow], 1);
    return;
  }
  const int64_t N = gl_words(level, A, k1, k, H, counters[kCntGDyn], lvl);
  const int kk = level == 1 ? k1 : k;    // a power of two
  const int ksh = __builtin_ctz((unsigned)kk);
  const int32_t kmask = kk - 1;
  const int64_t Rs = (N + kk - 1) >> ksh;
  const int64_t R0 = Rs + H;
  const int64_t limit = kL1 ? (rw_cap < kGlRidLimit - 1 ? rw_cap : kGlRidLimit - 1) : rw_cap;
  if (R0 > limit) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&counters[kCntGOverflow], 1);
    return;
  }
  // rulers opened by this level's walks are numbered from R0 on
  int32_t *dyn = level == 1 ? &counters[kCntGDyn] : &lvl[level];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < R0; q += stride) {
    int64_t e;
    if (q < Rs) {
      e = q << ksh;
    } else {
      const int32_t h = heads_in[q - Rs];
      const bool strided = (h & kmask) == 0;
      heads_out[q - Rs] = strided ? h >> ksh : (int32_t)q;
      if (strided) { rw_out[q] = kGlHole; continue; }
      e = h;
    }
    int64_t rid = q;
    // a walk longer than the level can only follow a cycle (malformed input):
    // it ends there, and a successor outside the level ends it too
    int64_t steps = 0;
    if (kL1) {
      int32_t *w = reinterpret_cast<int32_t *>(words);
      int32_t s = w[e];
      if (s == -2) { rw_out[rid] = kGlHole; continue; }
      uint32_t off = 0;   // weight walked since the ruler
      uint32_t len = 0;   // arcs walked since the ruler
      while (true) {
        w[e] = (int32_t)(((uint32_t)rid << kGlOffBits) | off);
        if (s < 0 || s >= N || ++steps > N) { rw_out[rid] = gl_pack(-1, off); break; }
        // weight of the successor
        const uint32_t ws = kW01 ? (uint32_t)(~__popc((uint32_t)s) & 1) : 1u;
        if ((s & kmask) == 0) { rw_out[rid] = gl_pack(s >> ksh, off + ws); break; }
        if (len == (uint32_t)kGlCap) {
          // open a ruler at s: the piece so far ends there
          const int64_t nr = R0 + atomicAdd(dyn, 1);
          if (nr >= limit) {
            atomicOr(&counters[kCntGOverflow], 1);
            rw_out[rid] = gl_pack(-1, off + ws);
            break;
          }
          rw_out[rid] = gl_pack((int32_t)nr, off + ws);
          rid = nr;
          off = 0;
          len = 0;
        } else {
          off += ws;
          ++len;
        }
        e = s;
        s = w[e];
      }
    } else {
      // 64-bit words (next, weight); codes (offset << 32 | ruler)
      uint64_t *w = reinterpret_cast<uint64_t *>(words);
      uint64_t cur = w[e];
      if (cur == kGlHole) { rw_out[rid] = kGlHole; continue; }
      uint32_t off = 0;
      int len = 0;
      // level 1 in this form (weighted arcs) keeps the level-1 cap
      const int cap = level == 1 ? kGlCap : kGlUpperCap;
      while (true) {
        const int32_t nx = (int32_t)(uint32_t)cur;
        const uint32_t wt = (uint32_t)(cur >> 32);
        w[e] = ((uint64_t)off << 32) | (uint32_t)rid;
        if (nx < 0 || nx >= N || ++steps > N) { rw_out[rid] = gl_pack(-1, off + wt); break; }
        if ((nx & kmask) == 0) { rw_out[rid] = gl_pack(nx >> ksh, off + wt); break; }
        if (++len == cap) {
          const int64_t nr = R0 + atomicAdd(dyn, 1);
          if (nr >= limit) {
            atomicOr(&counters[kCntGOverflow], 1);
            rw_out[rid] = gl_pack(-1, off + wt);
            break;
          }
          rw_out[rid] = gl_pack((int32_t)nr, off + wt);
          rid = nr;
          off = 0;
          len = 0;
        } else {
          off += wt;
        }
        e = nx;
        cur = w[e];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// top level: one workgroup, pointer jumping
// ---------------------------------------------------------------------------

// Words (next, w) of the top level become (-1, distance to the tail).  Up to
// kGlFinal words in LDS (barrier-separated rounds); a longer top level (more
// than about kGlFinal / 2 list heads) is jumped in place in global memory by
// the same workgroup: every version of a word read there is a true (next, w)
// pair, so a read of a word its owner is rewriting only speeds the jump up.
__global__ __launch_bounds__(kGlFinalThreads) void k_gfinal(int level, int64_t A, int k1, int k,
                                                            uint64_t *words, int32_t *counters,
                                                            const int32_t *lvl) {
  __shared__ uint64_t s_w[kGlFinal];
  __shared__ int s_more[3];
  if (counters[kCntGOverflow]) return;
  const int64_t H = counters[kCntGHeads];
  const int64_t N = gl_words(level, A, k1, k, H, counters[kCntGDyn], lvl);
  const int tid = threadIdx.x;
  if (tid == 0) {
    counters[kCntGTopWords] = (int32_t)N;
    s_more[0] = s_more[1] = s_more[2] = 0;
  }
  if (N <= kGlFinal) {
    const int m = (int)N;
    uint64_t ow[kGlFinalPer];
#pragma unroll
    for (int q = 0; q < kGlFinalPer; ++q) {
      const int i = tid + q * kGlFinalThreads;
      ow[q] = gl_pack(-1, 0);
      if (i < m) {
        const uint64_t v = words[i];
        const int32_t nx = (int32_t)(uint32_t)v;
        ow[q] = (v == kGlHole || nx >= m) ? gl_pack(-1, (uint32_t)(v >> 32)) : v;
        if (v == kGlHole) ow[q] = gl_pack(-1, 0);
        s_w[i] = ow[q];
      }
    }
    __syncthreads();
    for (int round = 0; round < 32; ++round) {
      bool more = false;
#pragma unroll
      for (int q = 0; q < kGlFinalPer; ++q) {
        const int32_t nx = (int32_t)(uint32_t)ow[q];
        if (nx >= 0) {
          const uint64_t nb = s_w[nx];
          ow[q] = gl_pack((int32_t)(uint32_t)nb, (uint32_t)(ow[q] >> 32) + (uint32_t)(nb >> 32));
          more |= (int32_t)(uint32_t)nb >= 0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kGlFinalPer; ++q) {
        const int i = tid + q * kGlFinalThreads;
        if (i < m) s_w[i] = ow[q];
      }
      if (more) s_more[round % 3] = 1;
      if (tid == 0) s_more[(round + 1) % 3] = 0;
      __syncthreads();
      if (!s_more[round % 3]) break;
    }
#pragma unroll
    for (int q = 0; q < kGlFinalPer; ++q) {
      const int i = tid + q * kGlFinalThreads;
      if (i < m) words[i] = ow[q];
    }
    return;
  }
  // long top level: in place in global memory (device-coherent accesses, so
  // that every round sees the words the others wrote before the barrier)
  for (int round = 0; round < 64; ++round) {
    bool more = false;
    for (int64_t i = tid; i < N; i += kGlFinalThreads) {
      const uint64_t v = __hip_atomic_load(&words[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int32_t nx = (int32_t)(uint32_t)v;
      if (nx >= 0 && nx < N) {
        const uint64_t nb = __hip_atomic_load(&words[nx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t nn = (int32_t)(uint32_t)nb;
        __hip_atomic_store(&words[i], gl_pack(nn, (uint32_t)(v >> 32) + (uint32_t)(nb >> 32)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        more |= nn >= 0;
      }
    }
    if (more) s_more[round % 3] = 1;
    if (tid == 0) s_more[(round + 1) % 3] = 0;
    __syncthreads();
    if (!s_more[round % 3]) break;
  }
  __syncthreads();
  for (int64_t i = tid; i < N; i += kGlFinalThreads)
    if (words[i] == kGlHole) words[i] = gl_pack(-1, 0);
}

// Codes of level `level` (>= 2) become distances: (-1, dist(ruler) - offset).
__global__ __launch_bounds__(kGlThreads) void k_gexpand(int level, int64_t A, int k1, int k,
                                                        uint64_t *words, const uint64_t *__restrict__ rw,
                                                        int64_t rw_cap,
                                                        const int32_t *__restrict__ counters,
                                                        const int32_t *__restrict__ lvl) {
  if (counters[kCntGOverflow]) return;
  const int64_t N = gl_words(level, A, k1, k, counters[kCntGHeads], counters[kCntGDyn], lvl);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += stride) {
    const uint64_t c = words[j];
    if (c == kGlHole) continue;
    const uint32_t rid = (uint32_t)c;
    if (rid >= rw_cap) continue;   // a word no walk reached (malformed input)
    const uint32_t dist = (uint32_t)(rw[rid] >> 32) - (uint32_t)(c >> 32);
    words[j] = gl_pack(-1, dist);
  }
}

// The level-1 rulers' distances, once ranked, as one 32-bit word each: the
// consumers below gather them at random (two per forest slot), and the
// compact array stays in an XCD's L2 far longer than the 64-bit words.
__global__ __launch_bounds__(kGlThreads) void k_gdist1(int64_t A, int k1,
                                                       const uint64_t *__restrict__ rw1,
                                                       int64_t rw1_cap, uint32_t *d1,
                                                       const int32_t *__restrict__ counters) {
  if (counters[kCntGOverflow]) return;
  int64_t R1 = (A + k1 - 1) / k1 + counters[kCntGHeads] + counters[kCntGDyn];
  if (R1 > rw1_cap) R1 = rw1_cap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < R1; j += stride)
    d1[j] = (uint32_t)(rw1[j] >> 32);
}

// distance to the tail of a level-1 arc from its code (0 for an arc no walk
// reached, which only malformed input leaves)
__device__ __forceinline__ uint32_t gl_arc_dist(int32_t code, const uint32_t *__restrict__ d1,
                                                int64_t rw1_cap) {
  const uint32_t c = (uint32_t)code;
  if ((int64_t)(c >> kGlOffBits) >= rw1_cap) return 0u;
  return d1[c >> kGlOffBits] - (c & (uint32_t)kGlCap);
}

// ---------------------------------------------------------------------------
// consumers of level 1
// ---------------------------------------------------------------------------

// Parent rule of Sec. III-D from both twin arcs' distances (the arc with the
// larger distance to the tail comes first and descends), plus, with cc, the
// default component roots and their count (as k_expand_parent).  Block 0
// copies the counters to host memory through host_out when given.
template <int B>
__global__ __launch_bounds__(B) void k_gparent(int64_t slots, int64_t n, const int32_t *__restrict__ tu,
                                               const int32_t *__restrict__ tv,
                                               const int32_t *__restrict__ w1,
                                               const uint32_t *__restrict__ d1, int64_t rw1_cap,
                                               const int32_t *__restrict__ cc,
                                               const int32_t *__restrict__ comp_root, int32_t *parent,
                                               int32_t *counters, int32_t *host_out) {
  if (host_out && blockIdx.x == 0 && threadIdx.x < kCntTotal)
    __hip_atomic_store(&host_out[threadIdx.x], counters[threadIdx.x], __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  if (counters[kCntGOverflow]) return;   // block-uniform: the caller ranks again
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < slots) {
    // the slot arrays stream through once: non-temporal loads leave the L2 to
    // d1, which every slot gathers from twice at random (C4: 475 -> 458 us)
    const int32_t a = __builtin_nontemporal_load(&tu[x]);
    if (a >= 0) {
      const int32_t b = __builtin_nontemporal_load(&tv[x]);
      const int64_t cw = __builtin_nontemporal_load(reinterpret_cast<const int64_t *>(w1) + x);
      const uint32_t da = gl_arc_dist((int32_t)(uint32_t)cw, d1, rw1_cap);
      const uint32_t db = gl_arc_dist((int32_t)(cw >> 32), d1, rw1_cap);
      if (da > db) parent[b] = a;   // a->b comes first in the tour: it descends
      else parent[a] = b;
    }
  }
  if (!cc) return;
  bool comp = false;
  if (x < n) {
    comp = cc[x] == (int32_t)x;
    if (comp && comp_root[x] == -1) parent[x] = (int32_t)x;
  }
  wave_count(comp, &counters[kCntComponents]);
}

__global__ __launch_bounds__(kGlThreads) void k_gdist(int64_t A, const int32_t *__restrict__ w1,
                                                      const uint32_t *__restrict__ d1,
                                                      int64_t rw1_cap, int32_t *dist,
                                                      const int32_t *__restrict__ counters) {
  if (counters[kCntGOverflow]) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < A) dist[e] = (int32_t)gl_arc_dist(w1[e], d1, rw1_cap);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

GlistPlan glist_plan(int64_t A, int64_t max_heads, int k1) {
  GlistPlan p;
  p.A = A;
  p.hcap = max_heads < kGlHeadCap ? (max_heads < 1 ? 1 : max_heads) : kGlHeadCap;
  // level-1 stride: as asked (0: 16, and 32 above 2^24 arcs, which keeps the
  // rulers' compact distances, gathered at random by the consumers, near the
  // size of one XCD's L2: on a 2^25-arc tour stride 32 cut the parent pass
  // 512 -> 478 us for a walk 1044 -> 1080 us; longer pieces make the walk
  // itself slower), doubled while the ruler ids would not fit 24 bits
  if (k1 <= 0) k1 = A > ((int64_t)1 << 24) ? 32 : 16;
  int s = 2;                         // a power of two, at least k1
  while (s < k1) s *= 2;
  while (s < 4096 && (A + s - 1) / s + A / kGlCap + p.hcap + 2 >= kGlRidLimit - 1) s *= 2;
  p.k1 = s;
  p.k = kGlStrideUpper;
  // level sizes without the heads decide the number of walk levels
  int64_t bound = A;                 // words of level L, heads aside
  int L = 1;
  p.cap[0] = 0;
  while (true) {
    const int kk = L == 1 ? p.k1 : p.k;
    const int64_t dynb = bound / (L == 1 ? kGlCap : kGlUpperCap) + 1;   // opened rulers
    const int64_t next_bound = (bound + kk - 1) / kk + dynb;
    // ruler words of level L (= words of level L + 1)
    p.cap[L] = next_bound + 2 * p.hcap + 2;
    bound = next_bound;
    ++L;
    if (bound <= (int64_t)kGlFinal * 3 / 4 || L >= kGlMaxLevels) break;
  }
  p.levels = L;   // walks at levels 1 .. L-1, the top (one workgroup) at level L
  return p;
}

size_t glist_ws_bytes(const GlistPlan &p) {
  size_t b = 2 * ws_bytes((size_t)p.hcap, 4) + ws_bytes(2 * kGlMaxLevels, 4) +
             ws_bytes((size_t)p.cap[1], 4);
  for (int L = 1; L < p.levels; ++L) b += ws_bytes((size_t)p.cap[L], 8);
  return b;
}

void glist_take(rst_ctx *ctx, const GlistPlan &p, GlistBufs &g) {
  g.plan = p;
  g.heads[0] = ws_take<int32_t>(ctx, (size_t)p.hcap);
  g.heads[1] = ws_take<int32_t>(ctx, (size_t)p.hcap);
  g.lvl = ws_take<int32_t>(ctx, 2 * kGlMaxLevels);
  for (int L = 1; L < p.levels; ++L) g.rw[L] = ws_take<uint64_t>(ctx, (size_t)p.cap[L]);
  g.d1 = ws_take<uint32_t>(ctx, (size_t)p.cap[1]);
}

static unsigned gl_grid(const rst_ctx *ctx, int64_t items) {
  // persistent-style grid: at most 8 workgroups of 256 per CU, fewer for
  // short levels (walkers loop over their rulers)
  const int64_t full = (int64_t)ctx->num_cus * 8;
  const int64_t want = (items + kGlThreads - 1) / kGlThreads;
  return (unsigned)(want < 1 ? 1 : (want < full ? want : full));
}

rst_status enqueue_glist_from_slots(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                                    const int32_t *tv, const int32_t *next,
                                    const int32_t *endsucc, const int32_t *head, int32_t *w1,
                                    GlistBufs &g, int32_t *counters) {
  const int64_t items = slots > n ? slots : n;
  RST_KMARK(ctx, RST_KERNEL_RANK_WORDS, 0);
  RST_SWEEP(ctx, k_gslot_words, items, slots, n, tu, tv, next, endsucc, head, w1, g.heads[0],
            g.plan.hcap, counters);
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_RANK_WORDS, 1);
  return RST_OK;
}

rst_status enqueue_glist_from_succ(rst_ctx *ctx, int64_t A, const int32_t *succ, int32_t *w1,
                                   uint8_t *haspred, GlistBufs &g, int32_t *counters) {
  RST_TRY(enqueue_fill(ctx, reinterpret_cast<int32_t *>(haspred), (A + 3) / 4, 0));
  hipLaunchKernelGGL(k_glist_words, dim3(grid_for(A, kGlThreads)), dim3(kGlThreads), 0, ctx->stream,
                     A, succ, w1, haspred);
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_glist_heads, dim3(grid_for(A, kGlThreads)), dim3(kGlThreads), 0, ctx->stream,
                     A, haspred, g.heads[0], g.plan.hcap, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_glist_rank(rst_ctx *ctx, void *w1, bool w1_wide, GlistBufs &g,
                              int32_t *counters, bool w01) {
  const GlistPlan &p = g.plan;
  RST_TRY(enqueue_fill(ctx, g.lvl, 2 * kGlMaxLevels, 0));   // rulers opened per level
  // walks, bottom up
  for (int L = 1; L < p.levels; ++L) {
    void *words = L == 1 ? w1 : static_cast<void *>(g.rw[L - 1]);
    // rulers of level L: about (words / stride) + heads
    const int64_t words_bound = L == 1 ? p.A : p.cap[L - 1];
    const int kk = L == 1 ? p.k1 : p.k;
    const unsigned grid = gl_grid(ctx, words_bound / kk + p.hcap);
    if (L == 1) {
      RST_KMARK(ctx, RST_KERNEL_RANK_WALK, 0);
      if (w1_wide)   // 64-bit (successor, weight) words at level 1 as well
        hipLaunchKernelGGL(k_gwalk<false>, dim3(grid), dim3(kGlThreads), 0, ctx->stream, L, p.A,
                           p.k1, p.k1, words, g.heads[0], g.heads[1], g.rw[1], p.cap[1], p.hcap,
                           counters, g.lvl);
      else if (w01)
        hipLaunchKernelGGL((k_gwalk<true, true>), dim3(grid), dim3(kGlThreads), 0, ctx->stream, L,
                           p.A, p.k1, p.k, words, g.heads[0], g.heads[1], g.rw[1], p.cap[1],
                           p.hcap, counters, g.lvl);
      else
        hipLaunchKernelGGL(k_gwalk<true>, dim3(grid), dim3(kGlThreads), 0, ctx->stream, L, p.A,
                           p.k1, p.k, words, g.heads[0], g.heads[1], g.rw[1], p.cap[1], p.hcap,
                           counters, g.lvl);
      RST_HIP(hipGetLastError());
      RST_KMARK(ctx, RST_KERNEL_RANK_WALK, 1);
    } else {
      hipLaunchKernelGGL(k_gwalk<false>, dim3(grid), dim3(kGlThreads), 0, ctx->stream, L, p.A,
                         p.k1, p.k, words, g.heads[(L - 1) & 1], g.heads[L & 1], g.rw[L], p.cap[L],
                         p.hcap, counters, g.lvl);
      RST_HIP(hipGetLastError());
    }
  }
  // the top level, then the codes of each level below it, top down
  hipLaunchKernelGGL(k_gfinal, dim3(1), dim3(kGlFinalThreads), 0, ctx->stream, p.levels, p.A, p.k1,
                     p.k, g.rw[p.levels - 1], counters, g.lvl);
  RST_HIP(hipGetLastError());
  for (int L = p.levels - 1; L >= 2; --L) {
    hipLaunchKernelGGL(k_gexpand, dim3(gl_grid(ctx, p.cap[L - 1])), dim3(kGlThreads), 0,
                       ctx->stream, L, p.A, p.k1, p.k, g.rw[L - 1], g.rw[L], p.cap[L], counters,
                       g.lvl);
    RST_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_gdist1, dim3(gl_grid(ctx, p.cap[1])), dim3(kGlThreads), 0, ctx->stream,
                     p.A, p.k1, g.rw[1], p.cap[1], g.d1, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_glist_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                                const int32_t *tv, const int32_t *w1, const GlistBufs &g,
                                const int32_t *cc, const int32_t *comp_root, int32_t *parent,
                                int32_t *counters, int32_t *host_out) {
  const int64_t items = (cc && n > slots) ? n : slots;
  if (cc) host_out = nullptr;   // the component count is only final after this pass
  RST_KMARK(ctx, RST_KERNEL_PARENT, 0);
  RST_SWEEP(ctx, k_gparent, items, slots, n, tu, tv, w1, g.d1, g.plan.cap[1], cc, comp_root,
            parent, counters, host_out);
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_PARENT, 1);
  return RST_OK;
}

rst_status enqueue_glist_dist(rst_ctx *ctx, int64_t A, const int32_t *w1, const GlistBufs &g,
                              int32_t *dist, const int32_t *counters) {
  hipLaunchKernelGGL(k_gdist, dim3(grid_for(A, kGlThreads)), dim3(kGlThreads), 0, ctx->stream, A,
                     w1, g.d1, g.plan.cap[1], dist, counters);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

}  // namespace rst

// ---------------------------------------------------------------------------
// last resort (more list heads or rulers than the buffers hold): Wyllie
// rounds over 64-bit (successor, hops) words of every arc
// ---------------------------------------------------------------------------
namespace rst {

template <int B>
__global__ __launch_bounds__(B) void k_gslot_words64(int64_t slots, const int32_t *__restrict__ tu,
                                                     const int32_t *__restrict__ tv,
                                                     const int32_t *__restrict__ next,
                                                     const int32_t *__restrict__ endsucc,
                                                     uint64_t *rank) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= slots) return;
  const int32_t a = tu[x];
  ulonglong2 out = make_ulonglong2(gl_pack(-1, 0), gl_pack(-1, 0));
  if (a >= 0) {
    const int32_t b = tv[x];
    const int2 nx = reinterpret_cast<const int2 *>(next)[x];
    const int32_t s0 = nx.y != -1 ? nx.y : endsucc[b];
    const int32_t s1 = nx.x != -1 ? nx.x : endsucc[a];
    out.x = gl_pack(s0, s0 >= 0 ? 1u : 0u);
    out.y = gl_pack(s1, s1 >= 0 ? 1u : 0u);
  }
  reinterpret_cast<ulonglong2 *>(rank)[x] = out;
}

template <int B>
__global__ __launch_bounds__(B) void k_wparent(int64_t slots, int64_t n, const int32_t *__restrict__ tu,
                                               const int32_t *__restrict__ tv,
                                               const uint64_t *__restrict__ rank,
                                               const int32_t *__restrict__ cc,
                                               const int32_t *__restrict__ comp_root, int32_t *parent,
                                               int32_t *counters) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < slots) {
    const int32_t a = tu[x];
    if (a >= 0) {
      const int32_t b = tv[x];
      const ulonglong2 r = reinterpret_cast<const ulonglong2 *>(rank)[x];
      if ((uint32_t)(r.x >> 32) > (uint32_t)(r.y >> 32)) parent[b] = a;
      else parent[a] = b;
    }
  }
  if (!cc) return;
  bool comp = false;
  if (x < n) {
    comp = cc[x] == (int32_t)x;
    if (comp && comp_root[x] == -1) parent[x] = (int32_t)x;
  }
  wave_count(comp, &counters[kCntComponents]);
}

rst_status glist_wyllie_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                               const int32_t *tv, const int32_t *next, const int32_t *endsucc,
                               uint64_t *rank, const int32_t *cc, const int32_t *comp_root,
                               int32_t *parent, int32_t *counters) {
  RST_SWEEP(ctx, k_gslot_words64, slots, slots, tu, tv, next, endsucc, rank);
  RST_HIP(hipGetLastError());
  RST_TRY(enqueue_rank_rounds(ctx, 2 * slots, rank, rank_rounds_for(2 * slots), nullptr, nullptr));
  const int64_t items = (cc && n > slots) ? n : slots;
  RST_SWEEP(ctx, k_wparent, items, slots, n, tu, tv, rank, cc, comp_root, parent, counters);
  RST_HIP(hipGetLastError());
  RST_TRY(enqueue_fill(ctx, counters + kCntGOverflow, 1, 0));
  return RST_OK;
}

}  // namespace rst
