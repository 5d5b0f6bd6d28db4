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

// bit k of the result set where byte k of the 32 bytes at b (0 or 1 each) is set
__device__ __forceinline__ uint32_t byte_flags32(const unsigned char *b) {
  const uint4 lo = *reinterpret_cast<const uint4 *>(b);
  const uint4 hi = *reinterpret_cast<const uint4 *>(b + 16);
  const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t x = w[k];
    r |= ((x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xfu) << (4 * k);
  }
  return r;
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

// Root marking fused with the end-of-list successors, for one designated root
// R = roots[0], after all hooks: a vertex roots its tree when it is R, or
// when it is its own parent (the minimum id of its component) and R lies in
// another component.  endsucc[v] is v's first out-arc, or -1 where v roots its
// tree (the cycle break), and such a v gets P[v] = v; the components are
// counted.  The labels are left as the hooks made them (the tour needs only
// the roots, which are final); the chain from R to its component's root is
// walked by every thread (the same few words, cached).
template <int B>
__global__ __launch_bounds__(B) void k_settle(int64_t n, const int32_t *__restrict__ roots,
                                                   const int32_t *__restrict__ cc,
                                                   const int32_t *__restrict__ head,
                                                   int32_t *endsucc, int32_t *parent,
                                                   int32_t *counters) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t R = roots[0];
  if (R < 0 || R >= n) {
    if (v == 0) atomicOr(&counters[kCntRangeErr], 1);
    return;
  }
  int32_t cR = R, nx;
  while (cR > (nx = cc[cR])) cR = nx;
  const bool comp_root = cc[v] == (int32_t)v;
  const bool tree_root = v == R || (comp_root && v != cR);
  endsucc[v] = tree_root ? -1 : head[v];
  if (tree_root) parent[v] = (int32_t)v;
  wave_count(comp_root, &counters[kCntComponents]);
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
constexpr int kRankPer = kRankTile / kRankThreads;     // 16 arcs (8 twin pairs) per thread
constexpr int kTileWalkSteps = 4;      // walk steps between two refills
constexpr bool kTileWaveShare = false; // rulers from the block's queue
constexpr int kTileAsync = 12;         // barrier-free jumping rounds before the synchronous ones
constexpr int kRankWaves = kRankThreads / 64;
constexpr int kRuler = 4;                              // every 4th arc starts a ruler
constexpr int kStrided = kRankTile / kRuler;           // 4096 strided rulers
constexpr int kPieceBits = 3;
constexpr int kPiece = 1 << kPieceBits;                // a walk opens a new ruler after 8 arcs
constexpr int kRulerSlots = 1 << (16 - kPieceBits);    // 8192: ruler ids fit the other 13 bits
constexpr int kMaxRulers = kRulerSlots - 1;            // id 8191 unused: its codes could read as -1
// static rulers (strided + segment heads) that leave room for every opened one
constexpr int kMaxStatic = kMaxRulers - kRankTile / kPiece;
// the 32-bit words of a 32-arc block whose arcs are off the stride
constexpr uint32_t kOffStride = kRuler == 4 ? 0xEEEEEEEEu : 0xFEFEFEFEu;
// LDS region of k_rank_tile: has-predecessor bits, ruler starts, ruler words
constexpr int kRegionBytes = 2 * (kMaxStatic + 1) + 4 * kRulerSlots;
static_assert(kRuler == 4 || kRuler == 8, "stride mask");

// Slot records of the tile pass over forest slots: for the twin arcs 2x and
// 2x+1 of slot x, the local id (in the arc tile) of the segment exit each one
// reaches and its hops to it, arc c in bits [32c, 32c + 28): exit | hops << 14.
// An exit reaches itself in 0 hops.  The successor of each exit goes to a
// second array beside the exits list.  The records take the first half of the
// rank buffer (A/2 words of 8 bytes), the successors its second half.
__device__ __forceinline__ uint32_t rec_half(int ex_local, uint32_t hops) {
  return (uint32_t)ex_local | (hops << 14);
}

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

// Within a tile: every segment head and every 4th arc starts a ruler.  One
// walk per ruler follows its piece of list in LDS to the next ruler, to the
// segment's exit, or for 8 arcs, where it opens a new ruler and goes on; every
// arc it passes is overwritten with (ruler << 3 | offset), so a single walk
// gives each arc its place.  Lanes of a wave take the rulers of the wave's
// share one after another as they become free (a wave costs the sum of its
// walks over 64 lanes, not 64 times its longest).  The rulers are then ranked
// by in-place pointer jumping on 32-bit words (last-ruler flag, the ruler
// reached -- or at the last ruler of a chain, the segment's exit -- and hops);
// an arc's (exit, hops) follows from its ruler's: the exit its chain ends at,
// and the ruler's hops less the arc's offset.  A tile with more
// segment heads than static ruler slots (no locality) is ranked by plain
// pointer jumping over all its arcs in LDS instead.
template <bool kFromSlots>
__global__ __launch_bounds__(kRankThreads, 8) void k_rank_tile(int64_t A, uint64_t *rank, int32_t *xid,
                                                            int32_t *exits, int32_t *tile_exits,
                                                            SlotSrc src) {
  // successor in the tile (-1 at an exit), then the arc's code; the last 64
  // entries are a spare slot per lane for idle lanes' accesses during the walk
  __shared__ int16_t ls[kRankTile + 64];
  __shared__ __align__(16) unsigned char region[kRegionBytes];   // rulers, or the fallback's hops
  __shared__ int s_extra, s_nexit, s_ndyn, s_qnext, s_or[3];
  int16_t *r_start = reinterpret_cast<int16_t *>(region);                  // [kMaxStatic + 1]
  uint32_t *r_word = reinterpret_cast<uint32_t *>(region + 2 * (kMaxStatic + 1));
  // until the walk, the ruler words' space holds one has-predecessor byte per arc
  unsigned char *haspred = reinterpret_cast<unsigned char *>(r_word);
  static_assert(kRegionBytes >= 2 * (kMaxStatic + 1) + 4 * kRulerSlots && 4 * kRulerSlots >= kRankTile &&
                (2 * (kMaxStatic + 1)) % 16 == 0 && kRegionBytes >= 2 * kRankTile,
                "ruler tables, predecessor bytes and fallback hops fit the region");
  uint16_t *dd = reinterpret_cast<uint16_t *>(region);                    // fallback: [kRankTile]

  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * kRankTile;
  const int cnt = (int)((A - e0) < kRankTile ? (A - e0) : kRankTile);
  if (tid == 0) { s_extra = 0; s_nexit = 0; s_ndyn = 0; s_qnext = 0; s_or[0] = s_or[1] = s_or[2] = 0; }
  for (int q = tid; q < kRankTile / 16; q += kRankThreads)
    reinterpret_cast<uint4 *>(haspred)[q] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  // Thread t takes the twin pairs p = t + k * kRankThreads (arcs 2p and 2p+1
  // of the tile), four pairs per half; the loads of a half are issued
  // together, then the end-of-list successors they need.
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    constexpr int P = kRankPer / 4;
    int32_t t[2 * P];                 // successor of each arc, -1 at a tail
    if (kFromSlots) {
      // successor of a->b: next(b->a), or at the end of b's list endsucc[b]
      int32_t dst[2 * P];
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const int i0 = 2 * (tid + (h * P + k) * kRankThreads);
        dst[2 * k] = dst[2 * k + 1] = -1;
        t[2 * k] = t[2 * k + 1] = -1;
        if (i0 < cnt) {   // cnt is even here: a slot's two arcs share a tile
          const int64_t x = (e0 + i0) >> 1;
          const int32_t a = src.tu[x];
          const int32_t b = src.tv[x];
          const int2 nx = reinterpret_cast<const int2 *>(src.next)[x];
          if (a >= 0) {
            dst[2 * k] = b;     t[2 * k] = nx.y;       // 2x = a->b, rev = 2x+1
            dst[2 * k + 1] = a; t[2 * k + 1] = nx.x;   // 2x+1 = b->a, rev = 2x
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 2 * P; ++q)
        if (dst[q] >= 0 && t[q] == -1) t[q] = src.endsucc[dst[q]];
#pragma unroll
      for (int q = 0; q < 2 * P; ++q)
        if (dst[q] < 0) t[q] = -1;
    } else {
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const int i0 = 2 * (tid + (h * P + k) * kRankThreads);
        t[2 * k] = t[2 * k + 1] = -1;
        if (i0 + 1 < cnt) {
          const ulonglong2 v = reinterpret_cast<const ulonglong2 *>(rank + e0)[i0 >> 1];
          t[2 * k] = (int32_t)(uint32_t)v.x;
          t[2 * k + 1] = (int32_t)(uint32_t)v.y;
        } else if (i0 < cnt) {
          t[2 * k] = (int32_t)(uint32_t)rank[e0 + i0];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int i0 = 2 * (tid + (h * P + k) * kRankThreads);
      uint32_t lv[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int i = i0 + c;
        bool is_exit = false;
        lv[c] = 0xffffu;
        if (i < cnt) {
          const int32_t sc = t[2 * k + c];
          const int64_t sl = (int64_t)sc - e0;
          if (sc >= 0 && sl >= 0 && sl < cnt) {
            lv[c] = (uint32_t)sl;
            haspred[sl] = 1;   // a plain byte store: an LDS atomic per arc serialises
          } else {
            is_exit = true;
          }
        }
        // exits of tile b go to exits[b*kRankTile + k], k from an LDS counter;
        // only exits are ever looked up in xid
        const int slot = wave_append(is_exit, &s_nexit);
        if (is_exit) {
          exits[e0 + slot] = (int32_t)(e0 + i);
          xid[e0 + i] = slot;
          if (kFromSlots) reinterpret_cast<int32_t *>(rank)[A + e0 + slot] = t[2 * k + c];
        }
      }
      if (i0 < cnt) *reinterpret_cast<uint32_t *>(&ls[i0]) = lv[0] | (lv[1] << 16);
    }
  }
  __syncthreads();
  // strided rulers own slots 0..kStrided-1; heads off the stride get the next ones
  for (int q = tid; q < kStrided; q += kRankThreads) r_start[q] = (int16_t)(q * kRuler);
  {
    // thread t < kRankTile / 32 reads the has-predecessor bytes of arcs
    // 32t..32t+31: arcs of the tile without a predecessor, off the stride
    uint32_t hb = 0u;
    if (tid < kRankTile / 32) {
      const int b0 = tid * 32;
      const uint32_t valid = b0 >= cnt ? 0u : (cnt - b0 >= 32 ? ~0u : (1u << (cnt - b0)) - 1u);
      hb = ~byte_flags32(haspred + b0) & valid & kOffStride;
    }
    const int c = __popc(hb);
    const int incl = wave_incl_scan(c);
    const int wtot = __shfl(incl, 63, 64);
    int base = 0;
    if ((tid & 63) == 63 && wtot) base = atomicAdd(&s_extra, wtot);
    int x = __shfl(base, 63, 64) + incl - c;
    while (hb) {
      const int bit = __ffs(hb) - 1;
      hb &= hb - 1u;
      if (kStrided + x < kMaxStatic) r_start[kStrided + x] = (int16_t)(tid * 32 + bit);
      ++x;
    }
  }
  __syncthreads();
  if (tid == 0) tile_exits[blockIdx.x] = s_nexit;
  const int nstatic = kStrided + s_extra;
  if (nstatic <= kMaxStatic) {
    // the walk: lanes take static rulers as they free up, from one queue of
    // the block (one LDS atomic per wave and refill: no wave idles while
    // another still has a share) or from their wave's own range
    constexpr int kWaves = kRankThreads / 64;
    const int share = (nstatic + kWaves - 1) / kWaves;
    int qnext = kTileWaveShare ? __builtin_amdgcn_readfirstlane(tid >> 6) * share : 0;
    const int qend = kTileWaveShare ? min(qnext + share, nstatic) : nstatic;
    bool more = qnext < qend;   // wave-uniform: the queue may hold rulers
    int q = -1, j = 0, len = 0;
    const int dummy = kRankTile + (tid & 63);
    while (true) {
      const uint64_t idle = __ballot(q < 0);
      if (more && idle != 0ull) {
        int base = qnext;
        if (!kTileWaveShare) {
          if ((tid & 63) == 0) base = atomicAdd(&s_qnext, (int)__popcll(idle));
          base = __shfl(base, 0, 64);
        }
        const int r = base + lanes_below(idle);
        if (q < 0 && r < qend) { q = r; j = r_start[r]; len = 0; }
        qnext = base + (int)__popcll(idle);
        more = qnext < qend;
      }
      if (__ballot(q >= 0) == 0ull) break;
      bool open = false;   // the piece reached kPiece arcs: continue as a new ruler
      // kTileWalkSteps steps per round of the wave-wide bookkeeping, written
      // with selects (idle lanes read and write their own spare entry)
#pragma unroll
      for (int rep = 0; rep < kTileWalkSteps; ++rep) {
        const bool act = q >= 0 && !open;
        const bool inr = j < cnt;          // a strided ruler past the end of a short tile ends at once
        const int jj = (act && inr) ? j : dummy;
        const int sj = ls[jj];
        const bool isexit = !inr || sj < 0;
        ls[jj] = isexit ? (int16_t)sj : (int16_t)((q << kPieceBits) | len);
        const int nj = sj & (kRankTile - 1);
        const bool str = !isexit && (nj & (kRuler - 1)) == 0;
        const int len1 = len + 1;
        const bool stop = act && (isexit || str);
        // a last ruler's word holds its exit in place of a next ruler
        const uint32_t rw = isexit ? (0x80000000u | ((uint32_t)(inr ? j : 0) << 16) | (uint32_t)len)
                                   : (((uint32_t)(nj / kRuler) << 16) | (uint32_t)len1);
        if (stop) r_word[q] = rw;
        const bool step = act && !isexit;
        open = open || (step && !str && len1 == kPiece);
        q = stop ? -1 : q;
        j = step ? nj : j;
        len = step ? len1 : len;
      }
      const int d = wave_append(open, &s_ndyn);
      if (open) {
        const int x = nstatic + d;
        if (x < kMaxRulers) {
          r_word[q] = ((uint32_t)x << 16) | (uint32_t)len;
          q = x;
          len = 0;
        } else {   // not reached on simple lists (at most kRankTile / kPiece are opened)
          r_word[q] = 0x80000000u | ((uint32_t)j << 16) | (uint32_t)len;
          q = -1;
        }
      }
    }
    __syncthreads();
    const int nrul = min(nstatic + s_ndyn, kMaxRulers);
    // pointer jumping over the rulers, in place: a word read while its owner
    // rewrites it is either version, and both are consistent (ruler, hops)
    // pairs.  First without barriers (each thread advances its own words on
    // whatever versions of the others' it finds, which only speeds the jumps
    // up) for at most kTileAsync rounds, then barrier-separated rounds finish,
    // usually in one.  Round flags rotate over three words so that one
    // barrier a round suffices: the flag cleared in a round was last read two
    // rounds earlier.
    constexpr int QP = kRulerSlots / kRankThreads;
    if (kTileAsync > 0) {
      uint32_t ownw[QP];
#pragma unroll
      for (int k = 0; k < QP; ++k) {
        const int r = tid + k * kRankThreads;
        ownw[k] = r < nrul ? r_word[r] : 0x80000000u;
      }
      for (int it = 0; it < kTileAsync; ++it) {
        bool pending = false;
#pragma unroll
        for (int k = 0; k < QP; ++k) {
          if (!(ownw[k] >> 31)) {
            const uint32_t w2 = __hip_atomic_load(&r_word[(ownw[k] >> 16) & (kRulerSlots - 1)],
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            ownw[k] = (w2 & 0xffff0000u) | ((ownw[k] + w2) & 0xffffu);
            __hip_atomic_store(&r_word[tid + k * kRankThreads], ownw[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
            pending |= !(ownw[k] >> 31);
          }
        }
        if (__ballot(pending) == 0ull) break;
      }
      __syncthreads();
    }
    for (int round = 0; round < 13; ++round) {
      bool pending = false;
#pragma unroll
      for (int k = 0; k < QP; ++k) {
        const int r = tid + k * kRankThreads;
        if (r < nrul) {
          const uint32_t w = r_word[r];
          if (!(w >> 31)) {
            const uint32_t w2 = r_word[(w >> 16) & (kRulerSlots - 1)];
            const uint32_t nw = (w2 & 0xffff0000u) | ((w + w2) & 0xffffu);
            r_word[r] = nw;
            pending |= !(nw >> 31);
          }
        }
      }
      if (pending) s_or[round % 3] = 1;
      if (tid == 0) s_or[(round + 1) % 3] = 0;
      __syncthreads();
      if (!s_or[round % 3]) break;
    }
    if (kFromSlots) {
      // one record per slot, coalesced: (exit, hops) of both twin arcs
#pragma unroll
      for (int k = 0; k < kRankPer / 2; ++k) {
        const int i0 = 2 * (tid + k * kRankThreads);
        if (i0 < cnt) {
          uint32_t half[2];
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const uint32_t code = (uint16_t)ls[i0 + c];
            half[c] = rec_half(i0 + c, 0u);
            if (code != 0xffffu) {
              const uint32_t w = r_word[code >> kPieceBits];
              half[c] = rec_half((w >> 16) & 0x3fffu, (w & 0xffffu) - (code & (kPiece - 1)));
            }
          }
          rank[(e0 + i0) >> 1] = ((uint64_t)half[1] << 32) | half[0];
        }
      }
      return;
    }
    // every arc but the exits: (exit of its chain, ruler hops - offset), coalesced
#pragma unroll
    for (int k = 0; k < kRankPer; ++k) {
      const int i = tid + k * kRankThreads;
      if (i < cnt) {
        const uint32_t c = (uint16_t)ls[i];
        if (c != 0xffffu) {
          const uint32_t w = r_word[c >> kPieceBits];
          rank[e0 + i] = pack_rank((int32_t)(e0 + ((w >> 16) & 0x3fffu)),
                                   (w & 0xffffu) - (c & (kPiece - 1)));
        }
      }
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
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
      const int i = tid + j * kRankThreads;
      if (i < cnt) {
        const int q = ls[i];
        np[j] = ls[q];
        nd[j] = (uint16_t)(dd[i] + dd[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {
      const int i = tid + j * kRankThreads;
      if (i < cnt) { ls[i] = np[j]; dd[i] = nd[j]; }
    }
    __syncthreads();   // fixed 15 rounds: enough for the 16384 arcs of a tile
  }
  if (kFromSlots) {
#pragma unroll
    for (int k = 0; k < kRankPer / 2; ++k) {
      const int i0 = 2 * (tid + k * kRankThreads);
      if (i0 < cnt)
        rank[(e0 + i0) >> 1] = ((uint64_t)rec_half(ls[i0 + 1], dd[i0 + 1]) << 32) |
                               rec_half(ls[i0], dd[i0]);
    }
    return;
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

// One workgroup ranks contracted lists of up to kSmallLds words (k_rank_small).
// For such lists the contraction writes each word packed in 32 bits: weighted
// hops (at most one tile's arcs, 17 bits) above the next word's index (15
// bits, kPkEnd at a tail); longer lists get 64-bit (next, hops) words for the
// multi-block rounds.
constexpr int kSmallThreads = 1024;
constexpr int kSmallPer = 19;
constexpr int kSmallLds = kSmallPer * kSmallThreads;    // 19456 words
constexpr uint32_t kPkEnd = 0x7fffu;
static_assert(kSmallLds < (int)kPkEnd && kRankTile < (1 << 17), "packed contracted words");

// Contracted list over the exits (one block per tile): next exit and weighted
// hops to it.  With kScan, every block first forms the exclusive prefix of the
// tiles' exit counts itself (up to kContractTiles tiles, in LDS) and block b
// stores base[b] (block 0 also base[tiles] = M), so no separate scan launch
// is needed; otherwise base comes from k_tile_scan.
constexpr int kContractTiles = 4096;
// kSlots: the tile pass wrote slot records (forest slots), else per-arc words.
template <bool kScan, bool kSlots>
__global__ __launch_bounds__(kBlock) void k_rank_contract(const int32_t *__restrict__ exits,
                                                          const int32_t *__restrict__ tile_exits,
                                                          int64_t *base, int64_t tiles, int64_t A,
                                                          const uint64_t *__restrict__ rank,
                                                          const int32_t *__restrict__ xid,
                                                          uint64_t *crank) {
  __shared__ int64_t s_base[kScan ? kContractTiles + 1 : 1];
  __shared__ int s_wave[kBlock / kWave];
  const int64_t *bs = base;
  if (kScan) {
    constexpr int PER = kContractTiles / kBlock;
    const int tid = threadIdx.x;
    int c[PER];
    int sum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = tid * PER + q;
      c[q] = t < tiles ? tile_exits[t] : 0;
      sum += c[q];
    }
    int total;
    int64_t run = block_excl_scan<kBlock>(sum, s_wave, &total);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      s_base[tid * PER + q] = run;
      run += c[q];
    }
    if (tid == 0) s_base[kContractTiles] = total;
    __syncthreads();
    if (tid == 0) {
      base[blockIdx.x] = s_base[blockIdx.x];
      if (blockIdx.x == 0) base[tiles] = total;
    }
    bs = s_base;
  }
  const int64_t e0 = (int64_t)blockIdx.x * kRankTile;
  const int cntb = tile_exits[blockIdx.x];
  const int64_t b0 = bs[blockIdx.x];
  const bool packed = bs[kScan ? kContractTiles : tiles] <= kSmallLds;   // M words in all
  uint32_t *cpk = reinterpret_cast<uint32_t *>(crank);
  for (int j = threadIdx.x; j < cntb; j += kBlock) {
    int32_t s, ex;
    uint32_t dl = 0;
    if (kSlots) {
      s = reinterpret_cast<const int32_t *>(rank)[A + e0 + j];   // the exit's successor
      if (s < 0) {
        if (packed) cpk[b0 + j] = kPkEnd;
        else crank[b0 + j] = pack_rank(-1, 0);
        continue;
      }
      const uint32_t h = (uint32_t)(rank[s >> 1] >> (32 * (s & 1)));
      const int sl = s & (kRankTile - 1);
      ex = s;                                  // s is an exit itself when it reaches itself
      if ((int)(h & 0x3fffu) != sl) {
        ex = (s & ~(kRankTile - 1)) + (int32_t)(h & 0x3fffu);
        dl = h >> 14;
      }
    } else {
      const int32_t x = exits[e0 + j];
      s = (int32_t)(uint32_t)rank[x];
      if (s < 0) {
        if (packed) cpk[b0 + j] = kPkEnd;
        else crank[b0 + j] = pack_rank(-1, 0);
        continue;
      }
      const uint64_t ws = rank[s];
      const int32_t id = (int32_t)(uint32_t)ws;
      ex = s;
      if (in_tile(id, s)) { ex = id; dl = (uint32_t)(ws >> 32); }
    }
    const int32_t nx = (int32_t)exit_index(ex, xid, bs);
    if (packed) cpk[b0 + j] = ((1u + dl) << 15) | (uint32_t)nx;
    else crank[b0 + j] = pack_rank(nx, 1u + dl);
  }
}

// The contracted list (M = base[tiles] words, packed (hops to the next word,
// next word)) ranked by one block, with no host round trip.  Like the tile
// pass: every 8th word and every list head starts a ruler; one walk per ruler
// follows its piece (opening a new ruler after 24 words), overwriting each
// word in place with (weighted distance from the ruler's start : 20, ruler :
// 12); the rulers are ranked by in-place pointer jumping on 64-bit words
// (last-ruler flag, next ruler, distance) and every word's distance to its
// tail follows.  Lists with too many heads for the ruler table (many small
// trees) are ranked by plain pointer jumping over all words in LDS instead.
// Longer lists (more than kSmallLds words; one CU would be slower on them
// than multi-block rounds) raise counters[kCntRankOverflow] and change
// nothing: the consumers then skip their work and the host ranks the list in
// multi-block rounds.  counters[kCntExits] = M, counters[kCntRankRounds] =
// pointer-jumping rounds.  Output: crank[i] = (-1, distance from word i to the
// tail of its list), 64-bit words over the packed input.
constexpr int kSmallRulers = 4096;
constexpr int kSmallPiece = 24;
constexpr int kSmallRuler = 8;                          // every 8th word starts a ruler
// LDS, ruler path: words uint32 [kSmallLds + 64] (the last 64 are a slot per
// lane for idle lanes' accesses), has-predecessor bytes [kSmallLds], ruler
// starts int16 [kSmallRulers], ruler words uint64 [kSmallRulers]; all-words
// path: (successor, hops) uint64 [kSmallLds].
constexpr int kSmOffHp = 4 * (kSmallLds + 64);
constexpr int kSmOffRs = kSmOffHp + kSmallLds;
constexpr int kSmOffRw = kSmOffRs + 2 * kSmallRulers;
constexpr int kSmBytes = (kSmOffRw + 8 * kSmallRulers) > 8 * kSmallLds ? (kSmOffRw + 8 * kSmallRulers)
                                                                       : 8 * kSmallLds;
static_assert(kSmOffHp % 16 == 0 && kSmallLds % 32 == 0 && kSmOffRw % 8 == 0, "ruler path LDS layout");
constexpr int kWalkSteps = 4;   // steps of every walk between two refills
constexpr bool kWaveShare = true;   // each wave walks its own range of static rulers
constexpr int kAsyncIters = 16;     // barrier-free jumping rounds before the synchronous ones

static_assert(kSmallRulers <= 4096 && kSmallPiece * kRankTile < (1 << 20), "walk word fields");
constexpr uint64_t kSmFinal = 1ull << 63;

__global__ __launch_bounds__(kSmallThreads) void k_rank_small(const int64_t *__restrict__ Mp,
                                                              uint64_t *crank, int64_t cap,
                                                              int32_t *counters) {
  __shared__ __align__(16) unsigned char s_raw[kSmBytes];
  __shared__ int s_extra, s_ndyn, s_qnext, s_or[3];
  const int tid = threadIdx.x;
  // the words are loaded before their count is known (cap = 64-bit words the
  // buffer holds), so that both loads overlap
  const uint32_t *cpk = reinterpret_cast<const uint32_t *>(crank);
  uint32_t own[kSmallPer];
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int i = tid + k * kSmallThreads;
    own[k] = i < 2 * cap ? cpk[i] : kPkEnd;
  }
  const int64_t M = *Mp;
  if (tid == 0) {
    counters[kCntExits] = (int32_t)M;
    s_extra = 0;
    s_ndyn = 0;
    s_qnext = 0;
    s_or[0] = s_or[1] = s_or[2] = 0;
  }
  if (M > kSmallLds) {
    if (tid == 0) counters[kCntRankOverflow] = 1;
    return;
  }
  const int m = (int)M;
  // out-of-range successors end the list; words past the list end at once
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k)
    if (tid + k * kSmallThreads >= m || (int)(own[k] & kPkEnd) >= m) own[k] |= kPkEnd;
  uint32_t *L = reinterpret_cast<uint32_t *>(s_raw);
  unsigned char *haspred = s_raw + kSmOffHp;
  int16_t *r_start = reinterpret_cast<int16_t *>(s_raw + kSmOffRs);
  uint64_t *r_word = reinterpret_cast<uint64_t *>(s_raw + kSmOffRw);
  for (int q = tid; q < kSmallLds / 16; q += kSmallThreads)
    reinterpret_cast<uint4 *>(haspred)[q] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  // plain byte stores mark the successors (an LDS atomic per word serialises)
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int i = tid + k * kSmallThreads;
    if (i < m) {
      const uint32_t t = own[k] & kPkEnd;
      L[i] = own[k];
      if (t != kPkEnd) haspred[t] = 1;
    }
  }
  __syncthreads();
  const int nstr = (m + kSmallRuler - 1) / kSmallRuler;
  for (int q = tid; q < nstr; q += kSmallThreads) r_start[q] = (int16_t)(q * kSmallRuler);
  // list heads off the 8-stride, read 32 words at a time from the bits
  for (int wd = tid; wd < (kSmallLds + 31) / 32; wd += kSmallThreads) {
    const int b0 = wd * 32;
    const uint32_t valid = b0 >= m ? 0u : (m - b0 >= 32 ? ~0u : (1u << (m - b0)) - 1u);
    uint32_t hb = ~byte_flags32(haspred + b0) & valid & 0xFEFEFEFEu;
    int x = hb ? atomicAdd(&s_extra, __popc(hb)) : 0;
    while (hb) {
      const int bit = __ffs(hb) - 1;
      hb &= hb - 1u;
      if (nstr + x < kSmallRulers) r_start[nstr + x] = (int16_t)(b0 + bit);
      ++x;
    }
  }
  __syncthreads();
  const int nstatic = nstr + s_extra;
  int rounds = 0;
  if (nstatic + (m + kSmallPiece - 1) / kSmallPiece <= kSmallRulers) {
    // the walk: lanes take the next static ruler as they free up, from their
    // wave's own range (no atomics; the ranges hold about equal work) or from
    // one queue of the block (one LDS atomic per wave and refill)
    constexpr int kWaves = kSmallThreads / 64;
    const int share = (nstatic + kWaves - 1) / kWaves;
    int qnext = kWaveShare ? __builtin_amdgcn_readfirstlane(tid >> 6) * share : 0;
    const int qend = kWaveShare ? min(qnext + share, nstatic) : nstatic;
    bool more = qnext < qend;
    int q = -1, j = 0, len = 0;
    uint32_t acc = 0;
    const int dummy = kSmallLds + (tid & 63);
    while (true) {
      const uint64_t idle = __ballot(q < 0);
      if (more && idle != 0ull) {
        int base = qnext;
        if (!kWaveShare) {
          if ((tid & 63) == 0) base = atomicAdd(&s_qnext, (int)__popcll(idle));
          base = __shfl(base, 0, 64);
        }
        const int r = base + lanes_below(idle);
        if (q < 0 && r < qend) { q = r; j = r_start[r]; len = 0; acc = 0; }
        qnext = base + (int)__popcll(idle);
        more = qnext < qend;
      }
      if (__ballot(q >= 0) == 0ull) break;
      bool open = false;
      // kWalkSteps steps per round of the wave-wide bookkeeping, written with
      // selects (idle lanes read and write their own spare word) so that the
      // steps need no branches
#pragma unroll
      for (int rep = 0; rep < kWalkSteps; ++rep) {
        const bool act = q >= 0 && !open;
        const int jj = act ? j : dummy;
        const uint32_t p = L[jj];
        L[jj] = (acc << 12) | ((uint32_t)q & (kSmallRulers - 1));
        const uint32_t t = p & kPkEnd;
        const bool end = t == kPkEnd;                       // the tail: last ruler of the chain
        const bool str = (t & (kSmallRuler - 1)) == 0;      // reaches the next static ruler
        const uint32_t nacc = acc + (p >> 15);
        const bool stop = act && (end || str);
        const uint32_t rw_hi = end ? (0x80000000u | (uint32_t)q) : t / kSmallRuler;
        const uint32_t rw_lo = end ? acc : nacc;
        if (stop) r_word[q] = ((uint64_t)rw_hi << 32) | rw_lo;
        open = open || (act && !end && !str && len == kSmallPiece - 1);
        q = stop ? -1 : q;
        j = act ? (int)t : j;
        acc = act ? nacc : acc;
        len = act ? len + 1 : len;
      }
      const int d = wave_append(open, &s_ndyn);
      if (open) {
        const int x = nstatic + d;
        if (x < kSmallRulers) {
          r_word[q] = ((uint64_t)x << 32) | acc;
          q = x;
          len = 0;
          acc = 0;
        } else {   // not reached on simple lists (at most m / kSmallPiece are opened)
          r_word[q] = kSmFinal | ((uint64_t)q << 32) | acc;
          q = -1;
        }
      }
    }
    __syncthreads();
    const int nrul = min(nstatic + s_ndyn, kSmallRulers);
    // pointer jumping over the rulers, in place (a word read while its owner
    // rewrites it is either version, both consistent).  First without
    // barriers: each thread advances its own words, reading whatever version
    // of the others' it finds (every version is a true (ruler reached,
    // distance) pair, so any interleaving only speeds the jumps up), for at
    // most kAsyncIters rounds; then barrier-separated rounds finish (three
    // rotating flags let one barrier a round suffice), usually in one.
    constexpr int QP = kSmallRulers / kSmallThreads;
    if (kAsyncIters > 0) {
      uint64_t ownw[QP];
#pragma unroll
      for (int k = 0; k < QP; ++k) {
        const int r = tid + k * kSmallThreads;
        ownw[k] = r < nrul ? r_word[r] : kSmFinal;
      }
      for (int it = 0; it < kAsyncIters; ++it) {
        ++rounds;
        bool pending = false;
#pragma unroll
        for (int k = 0; k < QP; ++k) {
          if (!(ownw[k] & kSmFinal)) {
            const uint64_t w2 = __hip_atomic_load(&r_word[(ownw[k] >> 32) & (kSmallRulers - 1)],
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            ownw[k] = (w2 & 0xffffffff00000000ull) | (uint32_t)((uint32_t)ownw[k] + (uint32_t)w2);
            __hip_atomic_store(&r_word[tid + k * kSmallThreads], ownw[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
            pending |= !(ownw[k] & kSmFinal);
          }
        }
        if (__ballot(pending) == 0ull) break;
      }
      __syncthreads();
    }
    for (int round = 0; round < 14; ++round) {
      bool pending = false;
#pragma unroll
      for (int k = 0; k < QP; ++k) {
        const int r = tid + k * kSmallThreads;
        if (r < nrul) {
          const uint64_t w = r_word[r];
          if (!(w & kSmFinal)) {
            const uint64_t w2 = r_word[(w >> 32) & (kSmallRulers - 1)];
            const uint64_t nw = (w2 & 0xffffffff00000000ull) | (uint32_t)((uint32_t)w + (uint32_t)w2);
            r_word[r] = nw;
            pending |= !(nw & kSmFinal);
          }
        }
      }
      ++rounds;
      if (pending) s_or[round % 3] = 1;
      if (tid == 0) s_or[(round + 1) % 3] = 0;
      __syncthreads();
      if (!s_or[round % 3]) break;
    }
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const int i = tid + k * kSmallThreads;
      if (i < m) {
        const uint32_t c = L[i];
        const uint32_t dist = (uint32_t)r_word[c & (kSmallRulers - 1)] - (c >> 12);
        crank[i] = pack_rank(-1, dist);
      }
    }
  } else {
    // all-words pointer jumping: each thread keeps its own words in registers
    // as 64-bit (next, hops); a round gathers the successors' words from LDS,
    // then (after a barrier) publishes its own.  ceil(log2 M) rounds suffice;
    // the cap also ends the loop on malformed (cyclic) input.
    int max_rounds = 1;
    while (((int64_t)1 << max_rounds) < M) ++max_rounds;
    uint64_t *s_word = reinterpret_cast<uint64_t *>(s_raw);
    uint64_t ow[kSmallPer];
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const uint32_t t = own[k] & kPkEnd;
      ow[k] = pack_rank(t == kPkEnd ? -1 : (int32_t)t, own[k] >> 15);
    }
    __syncthreads();   // every thread is done with the ruler tables
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const int i = tid + k * kSmallThreads;
      if (i < m) s_word[i] = ow[k];
    }
    __syncthreads();
    for (int round = 0; round < max_rounds; ++round) {
      bool more = false;
#pragma unroll
      for (int k = 0; k < kSmallPer; ++k) {
        const int32_t t = (int32_t)(uint32_t)ow[k];
        if (t >= 0) {
          const uint64_t nb = s_word[t];
          ow[k] = (((ow[k] >> 32) + (nb >> 32)) << 32) | (nb & 0xffffffffull);
          more |= (int32_t)(uint32_t)nb >= 0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kSmallPer; ++k) {
        const int i = tid + k * kSmallThreads;
        if (i < m) s_word[i] = ow[k];
      }
      ++rounds;
      if (more) s_or[round % 3] = 1;
      if (tid == 0) s_or[(round + 1) % 3] = 0;
      __syncthreads();
      if (!s_or[round % 3]) break;
    }
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const int i = tid + k * kSmallThreads;
      if (i < m) crank[i] = ow[k];
    }
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

// Distances of both arcs of a slot from its record (tile pass) and the
// contracted distances, then the parent rule; default component roots get
// P[v] = v and are counted (unless cc is null: done by k_settle).  With cc
// null the counters are final before this pass, and block 0 also copies them
// to host memory through host_out when given (system-scope stores), so that
// the call needs no copy after its last kernel.
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
                                                          int32_t *parent, int32_t *counters,
                                                          int32_t *host_out) {
  if (host_out && blockIdx.x == 0 && threadIdx.x < kCntTotal)
    __hip_atomic_store(&host_out[threadIdx.x], counters[threadIdx.x], __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  if (counters[kCntRankOverflow]) return;   // contracted list not ranked yet (block-uniform)
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < slots) {
    const int32_t a = tu[x];
    if (a >= 0) {
      const int32_t b = tv[x];
      // the slot record: exit and hops of both twin arcs; with one exit the
      // hops alone decide, else each adds its exit's contracted distance
      const uint64_t rec = rank[x];
      const uint32_t h0 = (uint32_t)rec, h1 = (uint32_t)(rec >> 32);
      uint32_t d0 = h0 >> 14, d1 = h1 >> 14;
      if ((h0 & 0x3fffu) != (h1 & 0x3fffu)) {
        const int64_t t0 = (2 * x) & ~(int64_t)(kRankTile - 1);
        d0 += (uint32_t)(crank[exit_index((int32_t)(t0 + (h0 & 0x3fffu)), xid, base)] >> 32);
        d1 += (uint32_t)(crank[exit_index((int32_t)(t0 + (h1 & 0x3fffu)), xid, base)] >> 32);
      }
      if (d0 > d1) parent[b] = a;   // a->b comes first in the tour: it descends
      else parent[a] = b;
    }
  }
  if (!cc) return;   // components' own parents and the count already done (k_settle)
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

rst_status enqueue_endsucc(rst_ctx *ctx, int64_t n, const int32_t *head, const int32_t *cc,
                           const int32_t *comp_root, int32_t *endsucc) {
  RST_SWEEP(ctx, k_endsucc, n, n, head, cc, comp_root, endsucc);
  RST_HIP(hipGetLastError());
  return RST_OK;
}

rst_status enqueue_settle(rst_ctx *ctx, int64_t n, const int32_t *roots, const int32_t *cc,
                          const int32_t *head, int32_t *endsucc, int32_t *parent,
                          int32_t *counters) {
  RST_KMARK(ctx, RST_KERNEL_SETTLE, 0);
  RST_SWEEP(ctx, k_settle, n, n, roots, cc, head, endsucc, parent, counters);
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_SETTLE, 1);
  return RST_OK;
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
    if (!from_slots->endsucc_ready)
      RST_TRY(enqueue_endsucc(ctx, from_slots->n, from_slots->head, from_slots->cc,
                              from_slots->comp_root, from_slots->endsucc));
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
  if (tiles <= kContractTiles) {
    if (from_slots)
      hipLaunchKernelGGL((k_rank_contract<true, true>), dim3((unsigned)tiles), dim3(kBlock), 0,
                         ctx->stream, rb.exits, rb.tile_exits, rb.tile_base, tiles, A, rank, xid,
                         rb.crank);
    else
      hipLaunchKernelGGL((k_rank_contract<true, false>), dim3((unsigned)tiles), dim3(kBlock), 0,
                         ctx->stream, rb.exits, rb.tile_exits, rb.tile_base, tiles, A, rank, xid,
                         rb.crank);
  } else {
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, ctx->stream, rb.tile_exits, tiles,
                       rb.tile_base);
    RST_HIP(hipGetLastError());
    if (from_slots)
      hipLaunchKernelGGL((k_rank_contract<false, true>), dim3((unsigned)tiles), dim3(kBlock), 0,
                         ctx->stream, rb.exits, rb.tile_exits, rb.tile_base, tiles, A, rank, xid,
                         rb.crank);
    else
      hipLaunchKernelGGL((k_rank_contract<false, false>), dim3((unsigned)tiles), dim3(kBlock), 0,
                         ctx->stream, rb.exits, rb.tile_exits, rb.tile_base, tiles, A, rank, xid,
                         rb.crank);
  }
  RST_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_rank_small, dim3(1), dim3(kSmallThreads), 0, ctx->stream,
                     rb.tile_base + tiles, rb.crank, (int64_t)rank_exit_capacity(A), counters);
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
                                 const int32_t *comp_root, int32_t *parent, int32_t *counters,
                                 int32_t *host_out) {
  const int64_t items = (cc && n > slots) ? n : slots;
  if (cc) host_out = nullptr;   // the component count is only final after this pass
  RST_KMARK(ctx, RST_KERNEL_PARENT, 0);
  RST_SWEEP(ctx, k_expand_parent, items, slots, n, tu, tv, rank, xid, tile_base, crank, cc,
            comp_root, parent, counters, host_out);
  RST_HIP(hipGetLastError());
  RST_KMARK(ctx, RST_KERNEL_PARENT, 1);
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
