// rst_internal.h -- shared declarations of the librst HIP sources (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "rst.h"

namespace rst {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per block for the sweep kernels

// Device scratch owned by a context: one buffer, bump-allocated per call.
struct Workspace {
  char *base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};

struct Options {
  int validate = 0;
  int bfs_levels_per_sync = 32;
  int bfs_grid = 0;
  int rank_elems_per_thread = 4;
  int heavy_degree = 1024;       // hooking: arcs of heavier vertices are chunked
  int sweep_block = 256;         // threads per block of the per-vertex/per-slot sweeps
  int bfs_heavy_degree = 1024;   // BFS: frontier vertices above this are split over blocks
  int graphs = 1;                // capture the device work of a call as a HIP graph and replay it
  int rank_stride = 0;           // sparse ruling set: every k-th arc starts a ruler
                                 // (0: 16, or 32 above 2^24 arcs)
  int hook_mode = 0;             // 0: by a locality probe, 1: vertex tiles, 2: global sweep
  int hook_sample = -1;          // global sweep: arcs each vertex hooks first (-1: by degree)
};

// Launch sweep kernel template `kern<B>` over `items` threads with the
// context's block size B (64, 128, 256, 512 or 1024).
#define RST_SWEEP(ctx, kern, items, ...)                                                        \
  do {                                                                                          \
    const int64_t it_ = (items);                                                                \
    switch ((ctx)->opt.sweep_block) {                                                           \
      case 64: hipLaunchKernelGGL(kern<64>, dim3(grid_for(it_, 64)), dim3(64), 0, (ctx)->stream, \
                                  __VA_ARGS__); break;                                          \
      case 128: hipLaunchKernelGGL(kern<128>, dim3(grid_for(it_, 128)), dim3(128), 0,            \
                                   (ctx)->stream, __VA_ARGS__); break;                          \
      case 512: hipLaunchKernelGGL(kern<512>, dim3(grid_for(it_, 512)), dim3(512), 0,            \
                                   (ctx)->stream, __VA_ARGS__); break;                          \
      case 1024: hipLaunchKernelGGL(kern<1024>, dim3(grid_for(it_, 1024)), dim3(1024), 0,        \
                                    (ctx)->stream, __VA_ARGS__); break;                         \
      default: hipLaunchKernelGGL(kern<256>, dim3(grid_for(it_, 256)), dim3(256), 0,             \
                                  (ctx)->stream, __VA_ARGS__); break;                           \
    }                                                                                           \
  } while (0)

struct Selector;
struct TuneCache;
struct GraphCache;

// batch.hip
rst_status enqueue_graph_mask(rst_ctx *ctx, const rst_batch *b, const uint8_t *method,
                              uint8_t *vmask);
// per vertex of a batch: 1 when its graph (a GConn+Euler one) is hooked by the
// global sweep -- most of a sample of its arcs leave their source's 8192-id
// tile -- else 0
rst_status enqueue_batch_hook_split(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                    const uint8_t *method, uint8_t *gsel);
rst_status enqueue_batch_check(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                               int32_t *counters);
rst_status enqueue_batch_arcs_check(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                    int32_t *counters);
rst_status enqueue_count_methods(rst_ctx *ctx, const rst_batch *b, const uint8_t *m,
                                 int32_t *counters);
rst_status enqueue_copy_u8(rst_ctx *ctx, const uint8_t *src, uint8_t *dst, int64_t count);
rst_status enqueue_single_batch(rst_ctx *ctx, const rst_csr *g, int32_t root, int64_t *vtx_off,
                                int64_t *arc_off, int32_t *roots);
rst_status enqueue_fill_u8(rst_ctx *ctx, uint8_t *dst, int64_t count, uint8_t value);

// selector.hip
size_t selector_scratch_bytes(const rst_ctx *ctx, const rst_csr *g, int32_t G);
rst_status run_selector(rst_ctx *ctx, const rst_csr *g, const rst_batch *b, uint8_t *choice);
void selector_free(rst_ctx *ctx);
const void *selector_weights(const rst_ctx *ctx);   // device weights of the loaded selector

}  // namespace rst

struct rst_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 256;
  rst::Workspace ws;
  rst::Options opt;
  hipEvent_t ev[36] = {};   // 0-6 stages, 8-31 kernel pairs, 32-35 batch marks
  int32_t *host_pinned = nullptr;   // small pinned host buffer for flag readback
  int32_t *host_pinned_dev = nullptr;   // its device address (null: read back by copies only)
  bool timing = false;              // record per-kernel events (a stats struct was passed)
  unsigned kev_mask = 0;            // kernel events recorded during the current call
  rst::Selector *selector = nullptr;
  rst::TuneCache *tune = nullptr;   // autotuned settings by graph class
  rst::GraphCache *graph = nullptr; // last captured graph of a call's device work
  hipStream_t cap_stream = nullptr; // private stream the capture runs on
};

namespace rst {

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
#define RST_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return RST_E_DEVICE;          \
  } while (0)

// per-kernel event pairs in ctx->ev[8..31], recorded only while ctx->timing is set
enum { kEvKernelBase = 8, kNumKernelTimes = 12, kEvBatchBase = 32, kNumEvents = 36 };
#define RST_KMARK(ctx, kernel, end)                                                          \
  do {                                                                                        \
    if ((ctx)->timing) {                                                                      \
      RST_HIP(hipEventRecord((ctx)->ev[kEvKernelBase + 2 * (kernel) + (end)], (ctx)->stream)); \
      (ctx)->kev_mask |= 1u << (2 * (kernel) + (end));                                        \
    }                                                                                         \
  } while (0)

#define RST_TRY(call)                                   \
  do {                                                  \
    rst_status s_ = (call);                             \
    if (s_ != RST_OK) return s_;                        \
  } while (0)

// Reserve `bytes` of workspace (256-byte aligned).  Grows the buffer (keeping
// nothing) only when called with ws.used == 0, i.e. at the start of a call.
rst_status ws_reserve(rst_ctx *ctx, size_t bytes);
template <class T>
T *ws_take(rst_ctx *ctx, size_t count) {
  size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
  char *p = ctx->ws.base + ctx->ws.used;
  ctx->ws.used += bytes;
  return reinterpret_cast<T *>(p);
}
inline size_t ws_bytes(size_t count, size_t elem) { return (count * elem + 255) & ~size_t(255); }

inline unsigned grid_for(int64_t items, int per_block) {
  int64_t g = (items + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// stage entry points (host side, enqueue only; defined in the .hip files)
// ---------------------------------------------------------------------------
struct ForestBufs {
  int32_t *cc;         // [n] union-find parents -> min-id labels
  int32_t *tu, *tv;    // [slots] recorded spanning edge per slot, -1 = empty
  int32_t *comp_root;  // [n] designated root of the component labelled v, or -1
  int32_t *counters;   // [64] device counters (see kCnt*)
  const uint8_t *vmask = nullptr;   // [n] nonzero: vertex excluded from hooking (nullable)
  // Euler arc lists built while hooking (nullable): every recorded edge of
  // slot x = (a, b) gives arcs 2x = a->b and 2x+1 = b->a, each put in front of
  // its source's list (head [n], next [2n]); the tile pass builds the lists of
  // its own edges in LDS, later hooks link with atomic exchanges.
  int32_t *head = nullptr;
  int32_t *next = nullptr;
  // Batches (global sweep): graph g owns vertices [vtx_off[g], vtx_off[g+1]);
  // giants[g] is the root of g's dominant tree or -1 ([num_graphs], written by
  // the hooking itself).  Without them the whole graph has one dominant tree
  // at most, counters[kCntGiant].
  const int64_t *vtx_off = nullptr;
  int32_t num_graphs = 0;
  int32_t *giants = nullptr;
  // Batches hooked graph by graph (nullable): per vertex 1 when its graph is
  // hooked by the global sweep, 0 when by the tile pass (which then runs
  // first and also initialises every vertex the sweep hooks).
  const uint8_t *gsel = nullptr;
};

enum {
  kCntChunks = 0,      // heavy-vertex chunk count (hooking)
  kCntRootErr = 1,     // two designated roots in one component
  kCntComponents = 2,  // vertices with cc[v] == v
  kCntRangeErr = 3,    // validation failure
  kCntBfsReached = 4,  // vertices reached by BFS
  kCntBfsLast = 5,     // deepest non-empty BFS level
  kCntCross = 6,       // cross-tile edges appended by the tile phase of hooking
  kCntExits = 7,       // segment exits of the tiled list ranking
  kCntBatchBfs = 8,    // graphs of a batch assigned to BFS
  kCntBatchBfsVtx = 9, // vertices of those graphs
  kCntCrossOverflow = 10,  // kept cross edges did not fit the LDS merge (fallback ran)
  kCntRankOverflow = 11,   // contracted list did not fit the one-block ranking
  kCntRankRounds = 12,     // pointer-jumping rounds of the contracted list
  kCntCrossDone = 13,      // the one-block merge of all kept edges succeeded
  kCntKept = 14,           // cross edges kept by the deduplication pass
  kCntKeptTop = 15,        // of those, the edges of the levels merged by the top pass
                           // (kCntKept and kCntKeptTop: one 8-byte word, added to at once)
  kCntGHeads = 16,         // sparse ruling set: list heads found
  kCntGDyn = 17,           //   rulers opened by walks that reached the piece cap
  kCntGOverflow = 18,      //   heads or ruler ids beyond capacity (caller ranks otherwise)
  kCntGTopWords = 19,      //   words of the top level (one workgroup)
  kCntDepthMax = 20,       // largest depth of a forest (rst_tree_depth)
  kCntPrHooks = 21,        // PR-RST: some edge joined two trees in this iteration
  kCntBatchArcErr = 22,    // validation: an arc of a batch leaves its graph
  kCntGiant = 23,          // global hooking: the dominant root after sampling, or -1
  kCntLocal = 24,          //   vertices whose first arc stays in their 8192-id tile
  kCntProbeArcs = 25,      // locality probe: sampled arcs
  kCntProbeCross = 26,     //   of those, arcs leaving their source's 8192-id tile
  kCntBccRoots = 27,       // biconnectivity: roots of the given parent array
  kCntBccItems = 29,       //   items of heavy vertices' arcs (not read back)
  kCntTotal = 28,          // counters read back after a call (the ones above)
};

// hook.hip
rst_status enqueue_fill(rst_ctx *ctx, int32_t *p, int64_t count, int32_t value);
// counters[0..31] = 0, counters[32] = root (the one-root buffer that follows them)
rst_status enqueue_reset_counters(rst_ctx *ctx, int32_t *counters, int32_t root);
rst_status enqueue_validate(rst_ctx *ctx, const rst_csr *g, int32_t *counters);
// cross: int2 [hook_cross_capacity], tile_cross: int32 [hook_tile_words], 8-byte aligned
rst_status enqueue_hook_csr(rst_ctx *ctx, const rst_csr *g, ForestBufs &f, int64_t *chunks,
                            int64_t chunk_cap, int2 *cross, int32_t *tile_cross);
size_t hook_cross_capacity(int64_t nnz);
size_t hook_tile_count(int64_t n);
int hook_level_count(int64_t n);
size_t hook_tile_words(int64_t n);   // int32 words of the tile_cross buffer
rst_status enqueue_hook_coo(rst_ctx *ctx, int64_t n, int64_t t, const int32_t *eu,
                            const int32_t *ev, int32_t *cc, int32_t *counters);
rst_status enqueue_compress(rst_ctx *ctx, int64_t n, int32_t *cc, int32_t *comp_root,
                            int32_t *head);
rst_status enqueue_count_roots(rst_ctx *ctx, int64_t n, const int32_t *cc, int32_t *counters);
size_t hook_chunk_capacity(const rst_ctx *ctx, int64_t nnz);

// ghook.hip: hooking by a sweep over the CSR in global memory (ids without
// locality): optional sampling of each vertex's first arcs, a dominant root,
// then the remaining arcs; fills f.cc, f.tu, f.tv (and the arc lists when
// f.head is set) like enqueue_hook_csr.  Needs nnz < 2^31.
// init false: every vertex was initialised by the tile pass (f.gsel batches)
rst_status enqueue_hook_global(rst_ctx *ctx, const rst_csr *g, ForestBufs &f, bool init = true);
int ghook_sample_arcs(const rst_ctx *ctx, const rst_csr *g);
// one workgroup samples arcs; counters[kCntProbeArcs], [kCntProbeCross] (zeroed
// by the caller beforehand) receive how many there were and how many left
// their 8192-id tile
rst_status enqueue_locality_probe(rst_ctx *ctx, const rst_csr *g, const uint8_t *vmask,
                                  int32_t *counters);

// euler.hip
// one designated root, after all hooks: the root's claim, end-of-list
// successors, the components' own parents and their count, in one pass
// (comp_root unused; the labels are not compressed)
rst_status enqueue_settle(rst_ctx *ctx, int64_t n, const int32_t *roots, const int32_t *cc,
                          const int32_t *head, int32_t *endsucc, int32_t *parent,
                          int32_t *counters);
rst_status enqueue_mark_roots(rst_ctx *ctx, const int32_t *roots, int32_t nroots, int64_t n,
                              const int32_t *cc, int32_t *comp_root, int32_t *parent,
                              int32_t *counters);
rst_status enqueue_link(rst_ctx *ctx, int64_t slots, const int32_t *tu, const int32_t *tv,
                        int32_t *head, int32_t *next);
rst_status enqueue_succ(rst_ctx *ctx, int64_t slots, const int32_t *tu, const int32_t *tv,
                        const int32_t *head, const int32_t *next, const int32_t *cc,
                        const int32_t *comp_root, uint64_t *rank);
rst_status enqueue_rank_init(rst_ctx *ctx, int64_t A, const int32_t *succ, uint64_t *rank);
rst_status enqueue_rank_rounds(rst_ctx *ctx, int64_t A, uint64_t *rank, int rounds,
                               hipEvent_t ev_begin, hipEvent_t ev_end);
rst_status enqueue_rank_extract(rst_ctx *ctx, int64_t A, const uint64_t *rank, int32_t *dist);
rst_status enqueue_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                          const int32_t *tv, const uint64_t *rank, const int32_t *cc,
                          const int32_t *comp_root, int32_t *parent, int32_t *counters);
int rank_rounds_for(int64_t max_list_len);
size_t rank_exit_capacity(int64_t A);
size_t rank_tile_count(int64_t A);
// Arcs given by forest slots: the tile pass computes each arc's successor
// itself (no separate successor pass).
struct SlotArcs {
  const int32_t *tu, *tv, *next, *head, *cc, *comp_root;
  int64_t n;          // vertices
  int32_t *endsucc;   // scratch [n]
  bool endsucc_ready = false;   // already filled (by enqueue_settle)
};
// Scratch of the tiled list ranking of A words: exits int32 [A+1], crank
// uint64 [A+1], tile_exits int32 [tiles], tile_base int64 [tiles+1].
struct RankBufs {
  int32_t *exits;
  uint64_t *crank;
  int32_t *tile_exits;
  int64_t *tile_base;
};
// Tiled list ranking of A words (succ, hops), with no host round trip: leaves
// (-1, distance to tail) in every word once the contracted list is ranked.
// from_slots: NULL -> rank[] already holds (succ, hops) words.  expand: expand
// here (otherwise the caller expands, e.g. fused with the parent rule).  When
// the contracted list was too long for the one-block ranking,
// counters[kCntRankOverflow] is set after the stream drains and every expand
// kernel has skipped its work: the caller then runs rank_overflow_fallback
// and expands again.
rst_status enqueue_rank_tiled(rst_ctx *ctx, int64_t A, uint64_t *rank, int32_t *xid,
                              const RankBufs &rb, int32_t *counters, const SlotArcs *from_slots,
                              bool expand);
rst_status enqueue_rank_expand(rst_ctx *ctx, int64_t A, uint64_t *rank, const int32_t *xid,
                               const RankBufs &rb, const int32_t *counters);
// multi-block rounds over the contracted list (M from the counters already read
// back to the host), then clears the overflow flag
rst_status rank_overflow_fallback(rst_ctx *ctx, const RankBufs &rb, int32_t *counters);
rst_status enqueue_expand_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                                 const int32_t *tv, const uint64_t *rank, const int32_t *xid,
                                 const int64_t *tile_base, const uint64_t *crank, const int32_t *cc,
                                 const int32_t *comp_root, int32_t *parent, int32_t *counters,
                                 int32_t *host_out = nullptr);

// glrank.hip: list ranking by a sparse ruling set in global memory (tours
// without id locality).  Level-1 words are int32 per arc (successor, then the
// arc's code); every later level is 64-bit (next, weight) words.
constexpr int kGlMaxLevels = 8;
constexpr int kGlStrideUpper = 16;   // ruler stride of the levels above the first
struct GlistPlan {
  int64_t A = 0;                      // level-1 words
  int64_t hcap = 1;                   // list heads the buffers hold
  int k1 = 16, k = kGlStrideUpper;    // ruler strides: level 1, the levels above
  int levels = 2;                     // walks at levels 1 .. levels-1, one workgroup at `levels`
  int64_t cap[kGlMaxLevels] = {};     // cap[L]: ruler words of level L
};
struct GlistBufs {
  GlistPlan plan;
  int32_t *heads[2] = {nullptr, nullptr};   // list heads per level (alternating)
  int32_t *lvl = nullptr;                   // [2 kGlMaxLevels]: rulers opened per level
  uint64_t *rw[kGlMaxLevels] = {};          // rw[L]: ruler words of level L
  uint32_t *d1 = nullptr;                   // [cap[1]]: each level-1 ruler's distance
                                            // to the tail (after the ranking)
};
// max_heads: an upper bound on the number of lists (capped internally)
GlistPlan glist_plan(int64_t A, int64_t max_heads, int k1);
size_t glist_ws_bytes(const GlistPlan &p);
void glist_take(rst_ctx *ctx, const GlistPlan &p, GlistBufs &g);
// level-1 words and list heads from forest slots (vertices with endsucc -1
// root their trees; their first out-arcs head the lists)
rst_status enqueue_glist_from_slots(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                                    const int32_t *tv, const int32_t *next,
                                    const int32_t *endsucc, const int32_t *head, int32_t *w1,
                                    GlistBufs &g, int32_t *counters);
// level-1 words and list heads from a successor array; haspred: A bytes scratch
rst_status enqueue_glist_from_succ(rst_ctx *ctx, int64_t A, const int32_t *succ, int32_t *w1,
                                   uint8_t *haspred, GlistBufs &g, int32_t *counters);
// w1: int32 level-1 words (unit weights; with w01 weight 1 on arc ids with an
// even number of one bits and 0 on the others), or with w1_wide uint64
// (successor, weight) words, whose
// codes become (offset << 32 | ruler)
rst_status enqueue_glist_rank(rst_ctx *ctx, void *w1, bool w1_wide, GlistBufs &g,
                              int32_t *counters, bool w01 = false);
rst_status enqueue_glist_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                                const int32_t *tv, const int32_t *w1, const GlistBufs &g,
                                const int32_t *cc, const int32_t *comp_root, int32_t *parent,
                                int32_t *counters, int32_t *host_out);
rst_status enqueue_glist_dist(rst_ctx *ctx, int64_t A, const int32_t *w1, const GlistBufs &g,
                              int32_t *dist, const int32_t *counters);
// last resort after counters[kCntGOverflow]: Wyllie rounds over every arc
// (rank: uint64 [2 slots]), the parent rule, and the flag cleared
rst_status glist_wyllie_parent(rst_ctx *ctx, int64_t slots, int64_t n, const int32_t *tu,
                               const int32_t *tv, const int32_t *next, const int32_t *endsucc,
                               uint64_t *rank, const int32_t *cc, const int32_t *comp_root,
                               int32_t *parent, int32_t *counters);
// end-of-list successors (one per vertex, -1 where the vertex roots its tree)
rst_status enqueue_endsucc(rst_ctx *ctx, int64_t n, const int32_t *head, const int32_t *cc,
                           const int32_t *comp_root, int32_t *endsucc);

// depth.hip: depth of every vertex of the forest given by parent (device),
// *max_depth (host, nullable) the largest; synchronous
rst_status run_tree_depth(rst_ctx *ctx, int64_t n, const int32_t *parent, int32_t *depth,
                          int64_t *max_depth);
// preorder numbers and subtree sizes of the tree given by parent (device),
// as records R[x] = (parent[x], pre(x), nd(x), 0); its buffers come from the
// workspace after the caller's (depth_ws_bytes less the counters); counters
// (device, 64) read back; synchronous
size_t depth_ws_bytes(int64_t n, const GlistPlan &p);
rst_status run_tour_preorder(rst_ctx *ctx, int64_t n, const int32_t *parent, int4 *R,
                             int32_t *counters);
// bcc.hip: biconnected components from a rooted spanning tree (synchronous)
rst_status run_biconnected(rst_ctx *ctx, const rst_csr *g, const int32_t *parent,
                           int32_t *arc_label, uint8_t *art, int64_t *num_components);

// prrst.hip: Path-Reversal RST of g rooted at root (synchronous; host loop)
rst_status run_pr_rst(rst_ctx *ctx, const rst_csr *g, int32_t root, int32_t *parent,
                      int64_t *iterations, int64_t *components);

// verify.hip: device check of a rooted spanning forest.  vc[0] += failures,
// vc[1] = min failing vertex (caller initialises 0 and INT32_MAX); anc0/anc1:
// int32 [n] scratch.
rst_status enqueue_verify(rst_ctx *ctx, const rst_csr *g, int32_t root, const int32_t *label,
                          const int32_t *parent, int32_t *anc0, int32_t *anc1, int32_t *vc);
// noalloc.hip: device address of the file-scope scratch of
// rst_components_noalloc, taken once per device (rst_create); the largest n
// that scratch holds
rst_status noalloc_init(int device);
int64_t noalloc_max_vertices();

// tune.hip
void tune_free(rst_ctx *ctx);
// api.hip
void graph_free(rst_ctx *ctx);

// bfs.hip
struct BfsBufs {
  int32_t *q[2];       // light frontier queues [n]
  int32_t *h[2];       // heavy frontier queues [heavy_cap]
  int32_t *cnt;        // [kBfsCntWords]: [3][2] rotating (light, heavy) counts, then the
                       // level state of the steps (see bfs.hip)
  int64_t heavy_cap;
};
constexpr int kBfsStateWord = 8;    // cnt[8..11]: level by launch parity, "wide next" by parity
constexpr int kBfsArcsWord = 12;    // cnt[12..14]: arcs of each rotating frontier slot
constexpr int kBfsCntWords = 16;
size_t bfs_heavy_capacity(const rst_ctx *ctx, int64_t n, int64_t nnz);
// level[] = -1 (and parent[] = -1 unless parent is NULL), counts zeroed
rst_status bfs_reset(rst_ctx *ctx, int64_t n, int32_t *level, int32_t *parent, BfsBufs &b);
// seed the level-0 frontier with a device list of roots; with gsel non-NULL
// only roots[g] with gsel[g] != 0 are seeded
rst_status bfs_seed_roots(rst_ctx *ctx, const rst_csr *g, const int32_t *roots, int32_t nroots,
                          int32_t *level, int32_t *parent, BfsBufs &b, int32_t *counters,
                          const uint8_t *gsel = nullptr);
// seed the level-0 frontier with every unreached vertex v that has cc[v] == v
// (and vsel[v] != 0 when vsel is non-NULL)
rst_status bfs_seed_unreached(rst_ctx *ctx, const rst_csr *g, const int32_t *cc, int32_t *level,
                              int32_t *parent, BfsBufs &b, int32_t *counters,
                              const uint8_t *vsel = nullptr);
// run levels until the frontier is empty; *levels_out = deepest level reached
// parent may be NULL (levels only); max_levels >= 0 caps the search
// enqueue `steps` level steps (rounded up to even) with no host
// synchronisation; every step expands at least one level until the search
// is done or max_levels is reached, so `steps` >= levels suffices
rst_status bfs_enqueue_steps(rst_ctx *ctx, const rst_csr *g, int32_t *level, int32_t *parent,
                             BfsBufs &b, int32_t *counters, int64_t steps, int64_t max_levels);
rst_status bfs_run_levels(rst_ctx *ctx, const rst_csr *g, int32_t *level, int32_t *parent,
                          BfsBufs &b, int32_t *counters, int64_t *levels_out,
                          int64_t max_levels = -1);

// batch.hip
rst_status enqueue_graph_mask(rst_ctx *ctx, const rst_batch *b, const uint8_t *method,
                              uint8_t *vmask);
rst_status enqueue_batch_check(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                               int32_t *counters);
rst_status enqueue_batch_arcs_check(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                    int32_t *counters);
rst_status enqueue_count_methods(rst_ctx *ctx, const rst_batch *b, const uint8_t *m,
                                 int32_t *counters);
rst_status enqueue_copy_u8(rst_ctx *ctx, const uint8_t *src, uint8_t *dst, int64_t count);
rst_status enqueue_fill_u8(rst_ctx *ctx, uint8_t *dst, int64_t count, uint8_t value);

// selector.hip
size_t selector_scratch_bytes(const rst_ctx *ctx, const rst_csr *g, int32_t G);
rst_status run_selector(rst_ctx *ctx, const rst_csr *g, const rst_batch *b, uint8_t *choice);
void selector_free(rst_ctx *ctx);

}  // namespace rst
