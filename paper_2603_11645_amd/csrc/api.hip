// api.hip -- the C ABI of librst (declared in include/rst.h): contexts, scratch
// management, argument checks and the host-side ordering of the stages.
#include "rst_internal.h"

#include <new>
#include <cstring>

namespace rst {

rst_status ws_reserve(rst_ctx *ctx, size_t bytes) {
  ctx->ws.used = 0;
  if (bytes <= ctx->ws.cap) return RST_OK;
  if (ctx->ws.base) {
    RST_HIP(hipStreamSynchronize(ctx->stream));
    RST_HIP(hipFree(ctx->ws.base));
    ctx->ws.base = nullptr;
    ctx->ws.cap = 0;
  }
  size_t cap = bytes + (bytes >> 3) + (1u << 20);
  if (hipMalloc(reinterpret_cast<void **>(&ctx->ws.base), cap) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws.base = nullptr;
    return RST_E_NOMEM;
  }
  ctx->ws.cap = cap;
  return RST_OK;
}

static rst_status check_csr(const rst_csr *g) {
  if (!g || g->n < 1 || g->nnz < 0 || !g->offsets) return RST_E_INVAL;
  if (g->nnz > 0 && !g->cols) return RST_E_INVAL;
  if (g->offset_bytes != 4 && g->offset_bytes != 8) return RST_E_INVAL;
  if (g->offset_bytes == 4 && g->nnz >= ((int64_t)1 << 31)) return RST_E_INVAL;
  // arc ids 2x+1 of the rooting stage are int32
  if (g->n >= ((int64_t)1 << 30)) return RST_E_INVAL;
  return RST_OK;
}

static rst_status read_counters(rst_ctx *ctx, const int32_t *counters) {
  RST_HIP(hipMemcpyAsync(ctx->host_pinned, counters, kCntTotal * sizeof(int32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  return RST_OK;
}

static rst_status run_validation(rst_ctx *ctx, const rst_csr *g, int32_t *counters) {
  if (!ctx->opt.validate) return RST_OK;
  RST_TRY(enqueue_validate(ctx, g, counters));
  RST_TRY(read_counters(ctx, counters));
  if (ctx->host_pinned[kCntRangeErr]) return RST_E_RANGE;
  return RST_OK;
}

// Elapsed time between two events of this call; a failed query (an event the
// call did not record) leaves no error behind for later hipGetLastError checks.
static bool event_ms(hipEvent_t a, hipEvent_t b, float *ms) {
  if (hipEventElapsedTime(ms, a, b) == hipSuccess) return true;
  (void)hipGetLastError();
  return false;
}

static void fill_stage_times(rst_ctx *ctx, rst_stats *st, const int *stage_of_gap, int nev) {
  float ms = 0.f;
  for (int i = 0; i + 1 < nev; ++i) {
    if (stage_of_gap[i] >= 0 && event_ms(ctx->ev[i], ctx->ev[i + 1], &ms))
      st->ms_stage[stage_of_gap[i]] += ms;
  }
  if (event_ms(ctx->ev[0], ctx->ev[nev - 1], &ms)) st->ms_total = ms;
}

// kernels whose two events were recorded during this call only
static void fill_kernel_times(rst_ctx *ctx, rst_stats *st) {
  for (int k = 0; k < kNumKernelTimes; ++k) {
    float ms = 0.f;
    if (((ctx->kev_mask >> (2 * k)) & 3u) != 3u) continue;
    if (event_ms(ctx->ev[kEvKernelBase + 2 * k], ctx->ev[kEvKernelBase + 2 * k + 1], &ms))
      st->ms_kernel[k] = ms;
  }
}

// enables per-kernel events for the duration of one API call
struct TimingScope {
  rst_ctx *ctx;
  TimingScope(rst_ctx *c, bool on) : ctx(c) { ctx->timing = on; ctx->kev_mask = 0; }
  ~TimingScope() { ctx->timing = false; }
};

static inline rst_status mark(rst_ctx *ctx, rst_stats *st, int i) {
  if (st) RST_HIP(hipEventRecord(ctx->ev[i], ctx->stream));
  return RST_OK;
}

static size_t rank_ws_bytes(int64_t A) {
  return ws_bytes(rank_exit_capacity(A), 4) + ws_bytes(rank_exit_capacity(A), 8) +
         ws_bytes(rank_tile_count(A), 4) + ws_bytes(rank_tile_count(A) + 1, 8);
}

static RankBufs take_rank_bufs(rst_ctx *ctx, int64_t A) {
  RankBufs r;
  r.exits = ws_take<int32_t>(ctx, rank_exit_capacity(A));
  r.crank = ws_take<uint64_t>(ctx, rank_exit_capacity(A));
  r.tile_exits = ws_take<int32_t>(ctx, rank_tile_count(A));
  r.tile_base = ws_take<int64_t>(ctx, rank_tile_count(A) + 1);
  return r;
}

// The ranking of the tour: per-tile in LDS (arc ids with locality, euler.hip)
// or by the sparse ruling set in global memory (glrank.hip).  Chosen from the
// hooking counters: when more than half as many edges crossed vertex tiles as
// there are vertices, the ids carry little locality and the tour leaves its
// tiles at almost every arc.
static bool prefer_sparse_rank(int64_t cross_edges, int64_t n) { return 2 * cross_edges > n; }

// Hooking variant of a call: the tile pass (hook.hip) or, for ids without
// locality, the global sweep (ghook.hip).  RST_OPT_HOOK_MODE 1 or 2 decides;
// in mode 0 one workgroup samples arcs, and when more than half of them leave
// their source's 8192-id tile the global sweep runs (one read-back of the
// counters, which the caller has zeroed).
static rst_status choose_hook(rst_ctx *ctx, const rst_csr *g, const uint8_t *vmask,
                              int32_t *counters, bool *global) {
  *global = false;
  if (g->nnz >= ((int64_t)1 << 31) || ctx->opt.hook_mode == 1) return RST_OK;
  if (ctx->opt.hook_mode == 2) { *global = true; return RST_OK; }
  RST_TRY(enqueue_fill(ctx, counters + kCntProbeArcs, 2, 0));
  RST_TRY(enqueue_locality_probe(ctx, g, vmask, counters));
  RST_TRY(read_counters(ctx, counters));
  *global = 2 * (int64_t)ctx->host_pinned[kCntProbeCross] > (int64_t)ctx->host_pinned[kCntProbeArcs];
  return RST_OK;
}

// After a replayed call (counters read back): whether the hooking and the
// ranking it captured still suit the data under its buffers.  The tile pass
// counts the edges that left their tiles, the global sweep the vertices whose
// first arc stayed in theirs.
static bool replay_wants_global(const rst_ctx *ctx, const rst_csr *g, bool global) {
  if (g->nnz >= ((int64_t)1 << 31) || ctx->opt.hook_mode == 1) return false;
  if (ctx->opt.hook_mode == 2) return true;
  if (global) return 2 * (int64_t)ctx->host_pinned[kCntLocal] < g->n;
  return 4 * (int64_t)ctx->host_pinned[kCntCross] > g->nnz;
}

static bool wants_sparse_rank(const rst_ctx *ctx, const rst_csr *g, bool global) {
  if (global) return 2 * (int64_t)ctx->host_pinned[kCntLocal] < g->n;
  return prefer_sparse_rank(ctx->host_pinned[kCntCross], g->n);
}

static rst_status enqueue_hook(rst_ctx *ctx, const rst_csr *g, ForestBufs &f, bool global,
                               int64_t *chunks, int64_t chunk_cap, int2 *cross,
                               int32_t *tile_cross) {
  if (f.gsel) {
    // a batch hooked graph by graph: the tile pass over the graphs with id
    // locality (it initialises every vertex, the others as singletons), then
    // the global sweep over the rest; no edge joins two graphs
    RST_TRY(enqueue_hook_csr(ctx, g, f, chunks, chunk_cap, cross, tile_cross));
    return enqueue_hook_global(ctx, g, f, false);
  }
  if (global) return enqueue_hook_global(ctx, g, f);
  return enqueue_hook_csr(ctx, g, f, chunks, chunk_cap, cross, tile_cross);
}

static GlistPlan gconn_glist_plan(const rst_ctx *ctx, int64_t n) {
  // lists: one per tree with an edge, at most n / 2
  return glist_plan(2 * n, n / 2 + 1, ctx->opt.rank_stride);
}

// Device buffers of one GConn+Euler run, taken from the workspace in a fixed
// order (the same pointers for the same graph size and workspace).
struct GconnWork {
  ForestBufs f;
  int64_t chunk_cap;
  int64_t *chunks;
  int2 *cross;
  int32_t *tile_cross;
  uint64_t *rank;
  int32_t *xid;
  int32_t *endsucc;
  bool settled = false;   // k_settle ran (one root): components' own parents and count done
  bool exported = false;  // the last kernel writes the counters to host_pinned (graph path)
  bool sparse = false;    // rank by the sparse ruling set (else per tile)
  bool sparse_ran = false;   // the sparse ruling set ran in this call (directly or as fallback)
  bool global_hook = false;  // hooking by the global sweep (else the tile pass)
  RankBufs rb;
  GlistBufs gl;
  int32_t *w1() const { return reinterpret_cast<int32_t *>(rank); }   // level-1 words alias rank
};

static GconnWork take_gconn_work(rst_ctx *ctx, const rst_csr *g, int32_t *counters,
                                 int32_t *cc_out, const uint8_t *vmask) {
  const int64_t n = g->n;
  GconnWork w;
  w.chunk_cap = (int64_t)hook_chunk_capacity(ctx, g->nnz);
  w.f.counters = counters;
  w.f.vmask = vmask;
  w.f.cc = cc_out ? cc_out : ws_take<int32_t>(ctx, n);
  w.f.tu = ws_take<int32_t>(ctx, n);
  w.f.tv = ws_take<int32_t>(ctx, n);
  w.f.comp_root = ws_take<int32_t>(ctx, n);
  // the arc lists are built while hooking (tile pass in LDS, later hooks by
  // atomic exchange), so no separate linking pass runs
  w.f.head = ws_take<int32_t>(ctx, n);
  w.f.next = ws_take<int32_t>(ctx, 2 * n);
  w.rank = ws_take<uint64_t>(ctx, 2 * n);
  w.chunks = ws_take<int64_t>(ctx, w.chunk_cap);
  w.cross = ws_take<int2>(ctx, hook_cross_capacity(g->nnz));
  w.tile_cross = ws_take<int32_t>(ctx, hook_tile_words(g->n));
  w.rb = take_rank_bufs(ctx, 2 * n);
  w.xid = ws_take<int32_t>(ctx, 2 * n);
  w.endsucc = ws_take<int32_t>(ctx, n);
  glist_take(ctx, gconn_glist_plan(ctx, n), w.gl);
  return w;
}

// Device work of the forest part (no host round trip): hooking, then either
// the one-root settle pass or compress + root marking.
static rst_status enqueue_gconn_forest(rst_ctx *ctx, const rst_csr *g, const int32_t *roots,
                                       int32_t nroots, int32_t *parent, rst_stats *st,
                                       GconnWork &w) {
  const int64_t n = g->n;
  RST_TRY(mark(ctx, st, 0));
  RST_TRY(enqueue_hook(ctx, g, w.f, w.global_hook, w.chunks, w.chunk_cap, w.cross, w.tile_cross));
  RST_TRY(mark(ctx, st, 1));
  w.settled = nroots == 1;
  if (w.settled) {
    // one pass: the root's claim, end-of-list successors, the components' own
    // parents and count (the labels are not needed further on this path; the
    // "roots" stage stays empty)
    RST_TRY(enqueue_settle(ctx, n, roots, w.f.cc, w.f.head, w.endsucc, parent, w.f.counters));
    RST_TRY(mark(ctx, st, 2));
    RST_TRY(mark(ctx, st, 3));
  } else {
    RST_TRY(enqueue_compress(ctx, n, w.f.cc, w.f.comp_root, nullptr));
    RST_TRY(mark(ctx, st, 2));
    RST_TRY(enqueue_mark_roots(ctx, roots, nroots, n, w.f.cc, w.f.comp_root, parent,
                               w.f.counters));
    RST_TRY(mark(ctx, st, 3));
  }
  return RST_OK;
}

// The sparse ruling set from the forest slots, then the parent rule.
static rst_status enqueue_gconn_sparse(rst_ctx *ctx, int64_t n, int32_t *parent, GconnWork &w,
                                       bool endsucc_ready, int32_t *host_out) {
  if (!endsucc_ready)
    RST_TRY(enqueue_endsucc(ctx, n, w.f.head, w.f.cc, w.f.comp_root, w.endsucc));
  RST_TRY(enqueue_glist_from_slots(ctx, n, n, w.f.tu, w.f.tv, w.f.next, w.endsucc, w.f.head,
                                   w.w1(), w.gl, w.f.counters));
  RST_TRY(enqueue_glist_rank(ctx, w.w1(), false, w.gl, w.f.counters));
  return enqueue_glist_parent(ctx, n, n, w.f.tu, w.f.tv, w.w1(), w.gl,
                              w.settled ? nullptr : w.f.cc, w.f.comp_root, parent, w.f.counters,
                              host_out);
}

// Device work of the rooting part (no host round trip): successors, ranking
// (per tile or sparse ruling set, as w.sparse says), parents.
static rst_status enqueue_gconn_rank(rst_ctx *ctx, const rst_csr *g, int32_t *parent,
                                     rst_stats *st, GconnWork &w) {
  const int64_t n = g->n;
  // with one root the counters are final before the parent pass, which then
  // also exports them when the call reads them that way
  int32_t *host_out = w.exported && w.settled ? ctx->host_pinned_dev : nullptr;
  // the successor pass is fused into the first ranking pass (stage "succ" stays empty)
  RST_TRY(mark(ctx, st, 4));
  if (w.sparse) {
    w.sparse_ran = true;
    if (!w.settled) RST_TRY(enqueue_endsucc(ctx, n, w.f.head, w.f.cc, w.f.comp_root, w.endsucc));
    RST_TRY(enqueue_glist_from_slots(ctx, n, n, w.f.tu, w.f.tv, w.f.next, w.endsucc, w.f.head,
                                     w.w1(), w.gl, w.f.counters));
    RST_TRY(enqueue_glist_rank(ctx, w.w1(), false, w.gl, w.f.counters));
    RST_TRY(mark(ctx, st, 5));
    RST_TRY(enqueue_glist_parent(ctx, n, n, w.f.tu, w.f.tv, w.w1(), w.gl,
                                 w.settled ? nullptr : w.f.cc, w.f.comp_root, parent,
                                 w.f.counters, host_out));
    RST_TRY(mark(ctx, st, 6));
    return RST_OK;
  }
  SlotArcs arcs{w.f.tu, w.f.tv, w.f.next, w.f.head, w.f.cc, w.f.comp_root, n, w.endsucc};
  arcs.endsucc_ready = w.settled;
  RST_TRY(enqueue_rank_tiled(ctx, 2 * n, w.rank, w.xid, w.rb, w.f.counters, &arcs, false));
  RST_TRY(mark(ctx, st, 5));
  // with one root, k_settle already set the components' own parents and counted them
  const int32_t *comp_cc = w.settled ? nullptr : w.f.cc;
  RST_TRY(enqueue_expand_parent(ctx, n, n, w.f.tu, w.f.tv, w.rank, w.xid, w.rb.tile_base,
                                w.rb.crank, comp_cc, w.f.comp_root, parent, w.f.counters,
                                host_out));
  RST_TRY(mark(ctx, st, 6));
  return RST_OK;
}

// Host side after the device work: read the counters (the call's one
// synchronisation), run a fallback ranking if one was flagged, fill the
// stats.  *components = components found.
static rst_status finish_gconn(rst_ctx *ctx, const rst_csr *g, int32_t *parent, rst_stats *st,
                               int64_t *components, GconnWork &w, bool *fallback = nullptr) {
  const int64_t n = g->n;
  int32_t *counters = w.f.counters;
  if (w.exported) RST_HIP(hipStreamSynchronize(ctx->stream));
  else RST_TRY(read_counters(ctx, counters));
  const bool rank_fallback = !w.sparse && ctx->host_pinned[kCntRankOverflow] != 0;
  if (rank_fallback) {
    // contracted list too long for the one-block ranking: rank the tour from
    // the slots by the sparse ruling set (the per-tile results are dropped)
    w.sparse_ran = true;
    RST_TRY(enqueue_fill(ctx, counters + kCntRankOverflow, 1, 0));
    RST_TRY(enqueue_gconn_sparse(ctx, n, parent, w, true, nullptr));
    RST_TRY(mark(ctx, st, 6));
    RST_TRY(read_counters(ctx, counters));
  }
  const bool last_resort = w.sparse_ran && ctx->host_pinned[kCntGOverflow] != 0;
  if (fallback) *fallback = rank_fallback || last_resort;
  if (last_resort) {
    // more list heads or rulers than the sparse ruling set holds
    RST_TRY(glist_wyllie_parent(ctx, n, n, w.f.tu, w.f.tv, w.f.next, w.endsucc, w.rank,
                                w.settled ? nullptr : w.f.cc, w.f.comp_root, parent, counters));
    RST_TRY(mark(ctx, st, 6));
    RST_TRY(read_counters(ctx, counters));
  }
  const int rounds = w.sparse_ran ? w.gl.plan.levels : ctx->host_pinned[kCntRankRounds];
  const int64_t exits_n =
      w.sparse_ran ? (2 * n + w.gl.plan.k1 - 1) / w.gl.plan.k1 + ctx->host_pinned[kCntGHeads] +
                         ctx->host_pinned[kCntGDyn]
                   : ctx->host_pinned[kCntExits];
  // the one-block merge of all levels is tried when there are more than 3 levels
  const bool groups =
      !w.global_hook && hook_level_count(n) > 3 && !ctx->host_pinned[kCntCrossDone];
  const int32_t paths =
      (!w.global_hook && ctx->host_pinned[kCntCrossOverflow] ? RST_PATH_CROSS_GLOBAL : 0) |
      (last_resort ? RST_PATH_RANK_GLOBAL : 0) | (groups ? RST_PATH_CROSS_GROUPS : 0) |
      (w.sparse_ran && !last_resort ? RST_PATH_RANK_SPARSE : 0) |
      (w.global_hook || w.f.gsel ? RST_PATH_HOOK_GLOBAL : 0) |
      ((w.global_hook || w.f.gsel) && ctx->host_pinned[kCntGiant] >= 0 ? RST_PATH_HOOK_GIANT : 0);
  if (ctx->host_pinned[kCntRangeErr]) return RST_E_INVAL;
  if (ctx->host_pinned[kCntRootErr]) return RST_E_INVAL;
  *components = ctx->host_pinned[kCntComponents];
  if (st) {
    static const int gaps[6] = {RST_STAGE_HOOK, RST_STAGE_COMPRESS, RST_STAGE_ARCS, RST_STAGE_SUCC,
                                RST_STAGE_RANK, RST_STAGE_PARENT};
    fill_stage_times(ctx, st, gaps, 7);
    fill_kernel_times(ctx, st);
    st->hook_rounds = w.global_hook ? (ghook_sample_arcs(ctx, g) > 0 ? 2 : 1)
                                    : 1 + hook_level_count(n);
    st->rank_rounds = rounds;
    st->rank_exits = exits_n;
    st->cross_edges = ctx->host_pinned[kCntCross];
    st->components = *components;
    st->method_used = RST_GCONN_EULER;
    st->paths = paths;
  }
  return RST_OK;
}

// GConn + Euler over the whole CSR, launched eagerly: the forest part, one
// read of the hooking counters to choose the ranking, the rooting part.
// Writes parent, returns the component count in *components; *sparse (host,
// nullable) receives the ranking chosen.
static rst_status run_gconn_euler_work(rst_ctx *ctx, const rst_csr *g, const int32_t *roots,
                                       int32_t nroots, int32_t *parent, rst_stats *st,
                                       int64_t *components, GconnWork &w, bool *sparse,
                                       bool *global_hook) {
  int32_t *counters = w.f.counters;
  // a batch hooked graph by graph decides on the device (f.gsel)
  if (w.f.gsel) w.global_hook = false;
  else RST_TRY(choose_hook(ctx, g, w.f.vmask, counters, &w.global_hook));
  if (global_hook) *global_hook = w.global_hook;
  RST_TRY(enqueue_gconn_forest(ctx, g, roots, nroots, parent, st, w));
  RST_TRY(read_counters(ctx, counters));
  w.sparse = w.f.gsel ? true : wants_sparse_rank(ctx, g, w.global_hook);
  if (sparse) *sparse = w.sparse;
  RST_TRY(enqueue_gconn_rank(ctx, g, parent, st, w));
  return finish_gconn(ctx, g, parent, st, components, w);
}

rst_status run_gconn_euler(rst_ctx *ctx, const rst_csr *g, const int32_t *roots, int32_t nroots,
                           int32_t *parent, rst_stats *st, int64_t *components,
                           int32_t *counters, int32_t *cc_out, const uint8_t *vmask = nullptr,
                           bool *sparse = nullptr, bool *global_hook = nullptr) {
  GconnWork w = take_gconn_work(ctx, g, counters, cc_out, vmask);
  return run_gconn_euler_work(ctx, g, roots, nroots, parent, st, components, w, sparse,
                              global_hook);
}

// ---------------------------------------------------------------------------
// captured HIP graphs of the device work of a call
// ---------------------------------------------------------------------------

// What a captured graph depends on: every pointer, size and value its kernels
// were launched with.
struct GraphKey {
  const void *offsets, *cols, *parent, *ws_base;
  int64_t n, nnz, ws_cap;
  int32_t offset_bytes, root;
  Options opt;
  // batch calls only (zero otherwise)
  const void *vtx_off, *arc_off, *roots, *method, *method_out, *selector;
  int32_t num_graphs, batch;
  bool operator==(const GraphKey &o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};

struct GraphCache {
  GraphKey key;
  hipGraphExec_t exec = nullptr;
  bool sparse = false;   // ranking captured for this key (sparse ruling set or per tile)
  bool global_hook = false;   // hooking captured for this key (global sweep or tile pass)
};

void graph_free(rst_ctx *ctx) {
  if (ctx->graph) {
    if (ctx->graph->exec) (void)hipGraphExecDestroy(ctx->graph->exec);
    delete ctx->graph;
    ctx->graph = nullptr;
  }
  if (ctx->cap_stream) {
    (void)hipStreamDestroy(ctx->cap_stream);
    ctx->cap_stream = nullptr;
  }
}

// Launch the device work `seq` on the context stream: replay the cached graph
// if its key matches, else capture `seq` (on a private stream, so that any
// user stream works) and launch the new graph.  Allocates nothing on the
// device outside the graph itself.
// Drop the captured graph (keeping the cache entry, now empty).
static void graph_forget(rst_ctx *ctx) {
  if (!ctx->graph) ctx->graph = new GraphCache;
  if (ctx->graph->exec) (void)hipGraphExecDestroy(ctx->graph->exec);
  ctx->graph->exec = nullptr;
  std::memset(&ctx->graph->key, 0, sizeof ctx->graph->key);
}

template <class Seq>
static rst_status run_graph(rst_ctx *ctx, const GraphKey &key, Seq seq) {
  if (ctx->graph && ctx->graph->exec && ctx->graph->key == key) {
    RST_HIP(hipGraphLaunch(ctx->graph->exec, ctx->stream));
    return RST_OK;
  }
  if (!ctx->graph) ctx->graph = new GraphCache;
  if (ctx->graph->exec) {
    RST_HIP(hipGraphExecDestroy(ctx->graph->exec));
    ctx->graph->exec = nullptr;
  }
  if (!ctx->cap_stream) RST_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  RST_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  hipStream_t user = ctx->stream;
  ctx->stream = ctx->cap_stream;
  const rst_status s = seq();
  ctx->stream = user;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
  if (s != RST_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return s != RST_OK ? s : RST_E_DEVICE;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  RST_HIP(ie);
  ctx->graph->exec = exec;
  ctx->graph->key = key;
  RST_HIP(hipGraphLaunch(exec, ctx->stream));
  return RST_OK;
}

static rst_status take_bfs_bufs(rst_ctx *ctx, const rst_csr *g, BfsBufs &b) {
  b.heavy_cap = (int64_t)bfs_heavy_capacity(ctx, g->n, g->nnz);
  b.q[0] = ws_take<int32_t>(ctx, g->n);
  b.q[1] = ws_take<int32_t>(ctx, g->n);
  b.h[0] = ws_take<int32_t>(ctx, b.heavy_cap);
  b.h[1] = ws_take<int32_t>(ctx, b.heavy_cap);
  b.cnt = ws_take<int32_t>(ctx, kBfsCntWords);
  return RST_OK;
}

static size_t bfs_ws_bytes(rst_ctx *ctx, const rst_csr *g) {
  const size_t hc = bfs_heavy_capacity(ctx, g->n, g->nnz);
  return 2 * ws_bytes(g->n, 4) + 2 * ws_bytes(hc, 4) + ws_bytes(kBfsCntWords, 4);
}

static size_t hook_ws_bytes(rst_ctx *ctx, const rst_csr *g) {
  return ws_bytes(hook_chunk_capacity(ctx, g->nnz), 8) + ws_bytes(hook_cross_capacity(g->nnz), 8) +
         ws_bytes(hook_tile_words(g->n), 4);
}

static size_t gconn_ws_bytes(rst_ctx *ctx, const rst_csr *g) {
  const size_t n = (size_t)g->n;
  return 6 * ws_bytes(n, 4) + 2 * ws_bytes(2 * n, 4) + ws_bytes(2 * n, 8) + hook_ws_bytes(ctx, g) +
         rank_ws_bytes(2 * g->n) + glist_ws_bytes(gconn_glist_plan(ctx, g->n));
}

// ---------------------------------------------------------------------------
// batches (Sec. III-D for every designated root of the packed forest)
// ---------------------------------------------------------------------------

// BFS steps enqueued in a captured batch call; a search still running after
// them is continued after the call's synchronisation
constexpr int kBatchBfsSteps = 16;

struct BatchWork {
  int32_t *counters = nullptr;
  uint8_t *m = nullptr;       // [G] method of each graph (1: BFS)
  uint8_t *vmask = nullptr;   // [n] 1 for the vertices of BFS graphs
  uint8_t *gsel = nullptr;    // [n] hooking graph by graph: 1 for the global sweep's graphs
  int32_t *level = nullptr;   // [n] BFS levels
  BfsBufs bb;
  GconnWork w;
  size_t sel_scratch = 0;     // workspace offset of the selector's scratch
};

// The device work of a batch call: checks, the method of every graph (given,
// chosen by the selector, or GConn+Euler), the vertex mask of the BFS graphs,
// GConn+Euler over the whole packed graph with those vertices masked (they
// stay singletons), then `bfs_steps` BFS steps from the roots of the BFS
// graphs, which overwrite the parents of their vertices.  No host round trip.
static rst_status enqueue_batch_device(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                       const uint8_t *method, int32_t *parent,
                                       uint8_t *method_out, BatchWork &bw, int64_t bfs_steps) {
  const int32_t G = b->num_graphs;
  const int64_t n = g->n;
  RST_TRY(enqueue_fill(ctx, bw.counters, 32, 0));
  RST_TRY(enqueue_batch_check(ctx, g, b, bw.counters));
  if (method) {
    RST_TRY(enqueue_copy_u8(ctx, method, bw.m, G));
  } else if (ctx->selector) {
    ctx->ws.used = bw.sel_scratch;
    RST_TRY(run_selector(ctx, g, b, bw.m));
  } else {
    RST_TRY(enqueue_fill_u8(ctx, bw.m, G, 0));
  }
  RST_TRY(enqueue_count_methods(ctx, b, bw.m, bw.counters));
  RST_TRY(enqueue_graph_mask(ctx, b, bw.m, bw.vmask));
  if (bw.w.f.gsel) RST_TRY(enqueue_batch_hook_split(ctx, g, b, bw.m, bw.gsel));
  RST_TRY(enqueue_gconn_forest(ctx, g, b->roots, G, parent, nullptr, bw.w));
  RST_TRY(enqueue_gconn_rank(ctx, g, parent, nullptr, bw.w));
  RST_TRY(bfs_reset(ctx, n, bw.level, nullptr, bw.bb));
  RST_TRY(bfs_seed_roots(ctx, g, b->roots, G, bw.level, parent, bw.bb, bw.counters, bw.m));
  RST_TRY(bfs_enqueue_steps(ctx, g, bw.level, parent, bw.bb, bw.counters, bfs_steps, -1));
  if (method_out) RST_TRY(enqueue_copy_u8(ctx, bw.m, method_out, G));
  return RST_OK;
}

// BFS of the batch's BFS graphs after their seeding (or after enqueued
// steps): levels until the frontier is empty; a disconnected BFS graph's other
// components are then searched from their minimum ids.
static rst_status batch_bfs_rest(rst_ctx *ctx, const rst_csr *g, int32_t *parent, BatchWork &bw,
                                 int64_t bfs_vertices, int64_t *levels) {
  RST_TRY(bfs_run_levels(ctx, g, bw.level, parent, bw.bb, bw.counters, levels));
  RST_TRY(read_counters(ctx, bw.counters));
  if (ctx->host_pinned[kCntBfsReached] >= bfs_vertices) return RST_OK;
  const int64_t n = g->n;
  // labels of the whole packed graph (seeds restricted to vertices of BFS
  // graphs); the GConn+Euler scratch is free again
  ForestBufs f;
  f.counters = bw.counters;
  f.cc = bw.w.f.cc;
  f.tu = bw.w.f.tu;
  f.tv = bw.w.f.tv;
  RST_TRY(enqueue_fill(ctx, bw.counters + kCntChunks, 1, 0));
  bool global_hook = false;
  RST_TRY(choose_hook(ctx, g, nullptr, bw.counters, &global_hook));
  RST_TRY(enqueue_hook(ctx, g, f, global_hook, bw.w.chunks, bw.w.chunk_cap, bw.w.cross,
                       bw.w.tile_cross));
  RST_TRY(enqueue_compress(ctx, n, f.cc, nullptr, nullptr));
  RST_TRY(bfs_seed_unreached(ctx, g, f.cc, bw.level, parent, bw.bb, bw.counters, bw.vmask));
  int64_t l2 = 0;
  return bfs_run_levels(ctx, g, bw.level, parent, bw.bb, bw.counters, &l2);
}

// After a replayed batch: one synchronisation (the GConn+Euler counters), the
// ranking fallbacks if flagged (they rewrite every parent, so the BFS graphs
// are searched again), the rest of the BFS if the enqueued steps did not
// finish it.
static rst_status finish_batch(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                               int32_t *parent, BatchWork &bw, rst_stats *st) {
  int64_t comps = 0;
  bw.w.sparse_ran = bw.w.sparse;
  bool reran = false;
  RST_TRY(finish_gconn(ctx, g, parent, nullptr, &comps, bw.w, &reran));
  if (ctx->host_pinned[kCntRangeErr]) return RST_E_INVAL;
  if (ctx->host_pinned[kCntBatchArcErr]) return RST_E_RANGE;
  const int32_t nbfs = ctx->host_pinned[kCntBatchBfs];
  const int64_t bfs_vertices = ctx->host_pinned[kCntBatchBfsVtx];
  if (nbfs == 0) return RST_OK;
  int64_t levels = 0;
  if (reran) {
    RST_TRY(enqueue_fill(ctx, bw.counters + kCntBfsReached, 1, 0));
    RST_TRY(bfs_reset(ctx, g->n, bw.level, nullptr, bw.bb));
    RST_TRY(bfs_seed_roots(ctx, g, b->roots, b->num_graphs, bw.level, parent, bw.bb, bw.counters,
                           bw.m));
  }
  RST_TRY(batch_bfs_rest(ctx, g, parent, bw, bfs_vertices, &levels));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  (void)st;
  return RST_OK;
}

// A batch call launched eagerly (first call with given buffers, stats or
// validation): the same stages with the host choosing the hooking and the
// ranking from device counters, and per-stage events when stats is set.
static rst_status run_batch_eager(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                  const uint8_t *method, int32_t *parent, uint8_t *method_out,
                                  rst_stats *stats, BatchWork &bw, bool *sparse,
                                  bool *global_hook) {
  const int32_t G = b->num_graphs;
  const int64_t n = g->n;
  int32_t *counters = bw.counters;
  RST_TRY(enqueue_fill(ctx, counters, 32, 0));
  RST_TRY(run_validation(ctx, g, counters));
  RST_TRY(enqueue_batch_check(ctx, g, b, counters));
  if (ctx->opt.validate) RST_TRY(enqueue_batch_arcs_check(ctx, g, b, counters));
  RST_TRY(mark(ctx, stats, kEvBatchBase));
  if (method) {
    RST_TRY(enqueue_copy_u8(ctx, method, bw.m, G));
  } else if (ctx->selector) {
    const size_t used = ctx->ws.used;
    ctx->ws.used = bw.sel_scratch;
    RST_TRY(run_selector(ctx, g, b, bw.m));
    ctx->ws.used = used;
  } else {
    RST_TRY(enqueue_fill_u8(ctx, bw.m, G, 0));
  }
  RST_TRY(mark(ctx, stats, kEvBatchBase + 1));
  RST_TRY(enqueue_count_methods(ctx, b, bw.m, counters));
  RST_TRY(read_counters(ctx, counters));
  if (ctx->host_pinned[kCntRangeErr]) return RST_E_INVAL;
  if (ctx->host_pinned[kCntBatchArcErr]) return RST_E_RANGE;
  const int32_t nbfs = ctx->host_pinned[kCntBatchBfs];
  const int64_t bfs_vertices = ctx->host_pinned[kCntBatchBfsVtx];
  RST_TRY(enqueue_graph_mask(ctx, b, bw.m, bw.vmask));
  if (bw.w.f.gsel) RST_TRY(enqueue_batch_hook_split(ctx, g, b, bw.m, bw.gsel));
  int64_t comps = 0;
  if (nbfs < G) {
    rst_stats inner;
    std::memset(&inner, 0, sizeof inner);
    RST_TRY(run_gconn_euler_work(ctx, g, b->roots, G, parent, stats ? &inner : nullptr, &comps,
                                 bw.w, sparse, global_hook));
    if (stats) {
      for (int i = 0; i < 8; ++i) stats->ms_stage[i] += inner.ms_stage[i];
      for (int i = 0; i < kNumKernelTimes; ++i) stats->ms_kernel[i] = inner.ms_kernel[i];
      stats->hook_rounds = inner.hook_rounds;
      stats->rank_rounds = inner.rank_rounds;
      stats->rank_exits = inner.rank_exits;
      stats->cross_edges = inner.cross_edges;
      stats->paths = inner.paths;
    }
  }
  int64_t levels = 0;
  if (nbfs > 0) {
    // multi-source BFS from the roots of the BFS graphs; parents of the other
    // graphs' vertices are left as written above
    RST_TRY(mark(ctx, stats, kEvBatchBase + 2));
    RST_TRY(bfs_reset(ctx, n, bw.level, nullptr, bw.bb));
    RST_TRY(bfs_seed_roots(ctx, g, b->roots, G, bw.level, parent, bw.bb, counters, bw.m));
    RST_TRY(batch_bfs_rest(ctx, g, parent, bw, bfs_vertices, &levels));
    RST_TRY(mark(ctx, stats, kEvBatchBase + 3));
  }
  if (method_out) RST_TRY(enqueue_copy_u8(ctx, bw.m, method_out, G));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  if (stats) {
    float ms = 0.f;
    if (event_ms(ctx->ev[kEvBatchBase], ctx->ev[kEvBatchBase + 1], &ms)) stats->ms_stage[RST_STAGE_SELECT] = ms;
    if (nbfs > 0 && event_ms(ctx->ev[kEvBatchBase + 2], ctx->ev[kEvBatchBase + 3], &ms)) stats->ms_stage[RST_STAGE_BFS] = ms;
    stats->ms_total = 0.f;
    for (int i = 0; i < 8; ++i) stats->ms_total += stats->ms_stage[i];
    stats->bfs_levels = levels;
    stats->components = comps;
    stats->method_used = nbfs == 0 ? RST_GCONN_EULER : (nbfs == G ? RST_BFS : -1);
  }
  return RST_OK;
}

}  // namespace rst

using namespace rst;

extern "C" {

rst_status rst_create(rst_ctx **out, int device, void *hip_stream) {
  if (!out) return RST_E_INVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return RST_E_INVAL;
  RST_HIP(hipSetDevice(device));
  rst_ctx *ctx = new (std::nothrow) rst_ctx();
  if (!ctx) return RST_E_NOMEM;
  ctx->device = device;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  // the allocation-free entry point's scratch address on this device
  if (noalloc_init(device) != RST_OK) {
    delete ctx;
    return RST_E_DEVICE;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0)
    ctx->num_cus = cus;
  for (int i = 0; i < kNumEvents; ++i) {
    if (hipEventCreate(&ctx->ev[i]) != hipSuccess) { rst_destroy(ctx); return RST_E_DEVICE; }
  }
  if (hipHostMalloc(reinterpret_cast<void **>(&ctx->host_pinned), 64 * sizeof(int32_t),
                    hipHostMallocDefault) != hipSuccess) {
    ctx->host_pinned = nullptr;
    rst_destroy(ctx);
    return RST_E_DEVICE;
  }
  if (hipHostGetDevicePointer(reinterpret_cast<void **>(&ctx->host_pinned_dev), ctx->host_pinned, 0) !=
      hipSuccess) {
    ctx->host_pinned_dev = nullptr;   // counters are then read back by copies
    (void)hipGetLastError();
  }
  *out = ctx;
  return RST_OK;
}

void rst_destroy(rst_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws.base) (void)hipFree(ctx->ws.base);
  for (int i = 0; i < kNumEvents; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  selector_free(ctx);
  tune_free(ctx);
  graph_free(ctx);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  delete ctx;
}

rst_status rst_set_stream(rst_ctx *ctx, void *hip_stream) {
  if (!ctx) return RST_E_INVAL;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return RST_OK;
}

rst_status rst_set_option(rst_ctx *ctx, rst_option opt, int64_t value) {
  if (!ctx) return RST_E_INVAL;
  switch (opt) {
    case RST_OPT_VALIDATE: ctx->opt.validate = value ? 1 : 0; return RST_OK;
    case RST_OPT_BFS_LEVELS_PER_SYNC:
      if (value < 1 || value > 4096) return RST_E_INVAL;
      ctx->opt.bfs_levels_per_sync = (int)value;
      return RST_OK;
    case RST_OPT_BFS_GRID:
      if (value < 0 || value > 65536) return RST_E_INVAL;
      ctx->opt.bfs_grid = (int)value;
      return RST_OK;
    case RST_OPT_RANK_ELEMS_PER_THREAD:
      if (value != 1 && value != 2 && value != 4 && value != 8) return RST_E_INVAL;
      ctx->opt.rank_elems_per_thread = (int)value;
      return RST_OK;
    case RST_OPT_HEAVY_DEGREE:
      if (value < 32 || value > (1 << 24)) return RST_E_INVAL;
      ctx->opt.heavy_degree = (int)value;
      return RST_OK;
    case RST_OPT_SWEEP_BLOCK:
      if (value != 64 && value != 128 && value != 256 && value != 512 && value != 1024)
        return RST_E_INVAL;
      ctx->opt.sweep_block = (int)value;
      return RST_OK;
    case RST_OPT_BFS_HEAVY_DEGREE:
      if (value < 32 || value > (1 << 24)) return RST_E_INVAL;
      ctx->opt.bfs_heavy_degree = (int)value;
      return RST_OK;
    case RST_OPT_GRAPHS:
      ctx->opt.graphs = value ? 1 : 0;
      return RST_OK;
    case RST_OPT_RANK_STRIDE:
      if (value != 0 && value != 4 && value != 8 && value != 16 && value != 32 && value != 64)
        return RST_E_INVAL;
      ctx->opt.rank_stride = (int)value;
      return RST_OK;
    case RST_OPT_HOOK_MODE:
      if (value < 0 || value > 2) return RST_E_INVAL;
      ctx->opt.hook_mode = (int)value;
      return RST_OK;
    case RST_OPT_HOOK_SAMPLE:
      if (value < -1 || value > 4) return RST_E_INVAL;
      ctx->opt.hook_sample = (int)value;
      return RST_OK;
  }
  return RST_E_INVAL;
}

rst_status rst_get_option(const rst_ctx *ctx, rst_option opt, int64_t *value) {
  if (!ctx || !value) return RST_E_INVAL;
  switch (opt) {
    case RST_OPT_VALIDATE: *value = ctx->opt.validate; return RST_OK;
    case RST_OPT_BFS_LEVELS_PER_SYNC: *value = ctx->opt.bfs_levels_per_sync; return RST_OK;
    case RST_OPT_BFS_GRID: *value = ctx->opt.bfs_grid; return RST_OK;
    case RST_OPT_RANK_ELEMS_PER_THREAD: *value = ctx->opt.rank_elems_per_thread; return RST_OK;
    case RST_OPT_HEAVY_DEGREE: *value = ctx->opt.heavy_degree; return RST_OK;
    case RST_OPT_SWEEP_BLOCK: *value = ctx->opt.sweep_block; return RST_OK;
    case RST_OPT_BFS_HEAVY_DEGREE: *value = ctx->opt.bfs_heavy_degree; return RST_OK;
    case RST_OPT_GRAPHS: *value = ctx->opt.graphs; return RST_OK;
    case RST_OPT_RANK_STRIDE: *value = ctx->opt.rank_stride; return RST_OK;
    case RST_OPT_HOOK_MODE: *value = ctx->opt.hook_mode; return RST_OK;
    case RST_OPT_HOOK_SAMPLE: *value = ctx->opt.hook_sample; return RST_OK;
  }
  return RST_E_INVAL;
}

rst_status rst_spanning_tree(rst_ctx *ctx, const rst_csr *g, int32_t root, rst_method method,
                             int32_t *parent, rst_stats *stats) {
  if (!ctx || !parent) return RST_E_INVAL;
  RST_TRY(check_csr(g));
  if (root < 0 || root >= g->n) return RST_E_INVAL;
  if (method != RST_GCONN_EULER && method != RST_BFS && method != RST_AUTO &&
      method != RST_PR_RST)
    return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  if (method == RST_PR_RST) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (ctx->opt.validate) {
      RST_TRY(ws_reserve(ctx, ws_bytes(64, 4)));
      int32_t *counters = ws_take<int32_t>(ctx, 64);
      RST_TRY(enqueue_fill(ctx, counters, 32, 0));
      RST_TRY(run_validation(ctx, g, counters));
    }
    RST_HIP(hipEventRecord(ctx->ev[0], ctx->stream));
    int64_t iters = 0, comps = 0;
    RST_TRY(run_pr_rst(ctx, g, root, parent, &iters, &comps));
    if (stats) {
      RST_HIP(hipEventRecord(ctx->ev[1], ctx->stream));
      RST_HIP(hipEventSynchronize(ctx->ev[1]));
      float ms = 0.f;
      if (event_ms(ctx->ev[0], ctx->ev[1], &ms)) stats->ms_total = ms;
      stats->hook_rounds = iters;
      stats->components = comps;
      stats->method_used = RST_PR_RST;
    }
    return comps > 1 ? RST_E_DISCONNECTED : RST_OK;
  }
  if (method == RST_AUTO) {
    // the selector's choice for this one graph (GConn+Euler without a selector)
    method = RST_GCONN_EULER;
    if (ctx->selector) {
      RST_TRY(ws_reserve(ctx, 3 * ws_bytes(2, 8) + ws_bytes(1, 1) + selector_scratch_bytes(ctx, g, 1)));
      int64_t *vtx_off = ws_take<int64_t>(ctx, 2);
      int64_t *arc_off = ws_take<int64_t>(ctx, 2);
      int32_t *roots = reinterpret_cast<int32_t *>(ws_take<int64_t>(ctx, 2));
      uint8_t *choice = ws_take<uint8_t>(ctx, 1);
      RST_TRY(enqueue_single_batch(ctx, g, root, vtx_off, arc_off, roots));
      const rst_batch one{1, vtx_off, arc_off, roots};
      RST_TRY(run_selector(ctx, g, &one, choice));
      uint8_t *hc = reinterpret_cast<uint8_t *>(ctx->host_pinned + 44);
      RST_HIP(hipMemcpyAsync(hc, choice, 1, hipMemcpyDeviceToHost, ctx->stream));
      RST_HIP(hipStreamSynchronize(ctx->stream));
      if (*hc) method = RST_BFS;
    }
  }
  if (stats) std::memset(stats, 0, sizeof(*stats));
  TimingScope timing(ctx, stats != nullptr);

  size_t bytes = ws_bytes(64, 4) + gconn_ws_bytes(ctx, g);
  if (method == RST_BFS) bytes += bfs_ws_bytes(ctx, g) + ws_bytes(g->n, 4);
  RST_TRY(ws_reserve(ctx, bytes));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  int32_t *rootbuf = counters + 32;

  if (method == RST_GCONN_EULER && ctx->opt.graphs && !stats && !ctx->opt.validate) {
    // the whole device part of the call as one captured graph, replayed while
    // the graph, buffers and settings stay the same
    GraphKey key;
    std::memset(&key, 0, sizeof key);
    key.offsets = g->offsets; key.cols = g->cols; key.parent = parent;
    key.ws_base = ctx->ws.base; key.ws_cap = (int64_t)ctx->ws.cap;
    key.n = g->n; key.nnz = g->nnz; key.offset_bytes = g->offset_bytes; key.root = root;
    key.opt = ctx->opt;
    int64_t comps = 0;
    if (!ctx->graph || !(ctx->graph->key == key)) {
      // first call with these buffers and settings: run eagerly, choosing the
      // ranking from the hooking counters; the next call captures that choice
      RST_TRY(enqueue_reset_counters(ctx, counters, root));
      bool sparse = false, global_hook = false;
      RST_TRY(run_gconn_euler(ctx, g, rootbuf, 1, parent, nullptr, &comps, counters, nullptr,
                              nullptr, &sparse, &global_hook));
      graph_forget(ctx);
      ctx->graph->key = key;
      ctx->graph->sparse = sparse;
      ctx->graph->global_hook = global_hook;
      return comps > 1 ? RST_E_DISCONNECTED : RST_OK;
    }
    GconnWork w = take_gconn_work(ctx, g, counters, nullptr, nullptr);
    w.settled = true;   // one root (a replay does not run the host code of the enqueue functions)
    w.exported = ctx->host_pinned_dev != nullptr;
    w.sparse = ctx->graph->sparse;
    w.global_hook = ctx->graph->global_hook;
    RST_TRY(run_graph(ctx, key, [&]() -> rst_status {
      RST_TRY(enqueue_reset_counters(ctx, counters, root));
      RST_TRY(enqueue_gconn_forest(ctx, g, rootbuf, 1, parent, nullptr, w));
      return enqueue_gconn_rank(ctx, g, parent, nullptr, w);
    }));
    w.sparse_ran = w.sparse;
    RST_TRY(finish_gconn(ctx, g, parent, nullptr, &comps, w));
    // the data under these buffers may have changed since the capture: when
    // the other hooking or ranking suits it now, the next call captures that
    const bool want_global = replay_wants_global(ctx, g, w.global_hook);
    const bool want_sparse = want_global == w.global_hook
                                 ? wants_sparse_rank(ctx, g, w.global_hook)
                                 : want_global;
    if ((want_sparse != w.sparse || want_global != w.global_hook) && ctx->graph->exec) {
      RST_HIP(hipGraphExecDestroy(ctx->graph->exec));
      ctx->graph->exec = nullptr;
      ctx->graph->sparse = want_sparse;
      ctx->graph->global_hook = want_global;
    }
    return comps > 1 ? RST_E_DISCONNECTED : RST_OK;
  }

  RST_TRY(enqueue_reset_counters(ctx, counters, root));
  RST_TRY(run_validation(ctx, g, counters));

  if (method == RST_GCONN_EULER) {
    int64_t comps = 0;
    RST_TRY(run_gconn_euler(ctx, g, rootbuf, 1, parent, stats, &comps, counters, nullptr));
    return comps > 1 ? RST_E_DISCONNECTED : RST_OK;
  }

  // BFS from root; unreached components (if any) are then rooted at their
  // minimum id by a second multi-source search.
  BfsBufs b;
  RST_TRY(take_bfs_bufs(ctx, g, b));
  int32_t *level = ws_take<int32_t>(ctx, g->n);
  RST_TRY(mark(ctx, stats, 0));
  RST_TRY(bfs_reset(ctx, g->n, level, parent, b));
  RST_TRY(bfs_seed_roots(ctx, g, rootbuf, 1, level, parent, b, counters));
  int64_t levels = 0;
  RST_TRY(bfs_run_levels(ctx, g, level, parent, b, counters, &levels));
  RST_TRY(mark(ctx, stats, 1));
  RST_TRY(read_counters(ctx, counters));
  const int64_t reached = ctx->host_pinned[kCntBfsReached];
  rst_status status = RST_OK;
  int64_t comps = 1;
  if (reached < g->n) {
    ForestBufs f;
    f.counters = counters;
    f.cc = ws_take<int32_t>(ctx, g->n);
    f.tu = ws_take<int32_t>(ctx, g->n);
    f.tv = ws_take<int32_t>(ctx, g->n);
    const int64_t chunk_cap = (int64_t)hook_chunk_capacity(ctx, g->nnz);
    int64_t *chunks = ws_take<int64_t>(ctx, chunk_cap);
    int2 *cross = ws_take<int2>(ctx, hook_cross_capacity(g->nnz));
    int32_t *tile_cross = ws_take<int32_t>(ctx, hook_tile_words(g->n));
    bool global_hook = false;
    RST_TRY(choose_hook(ctx, g, f.vmask, f.counters, &global_hook));
    RST_TRY(enqueue_hook(ctx, g, f, global_hook, chunks, chunk_cap, cross, tile_cross));
    RST_TRY(enqueue_compress(ctx, g->n, f.cc, nullptr, nullptr));
    RST_TRY(enqueue_count_roots(ctx, g->n, f.cc, counters));
    RST_TRY(bfs_seed_unreached(ctx, g, f.cc, level, parent, b, counters));
    int64_t l2 = 0;
    RST_TRY(bfs_run_levels(ctx, g, level, parent, b, counters, &l2));
    RST_TRY(read_counters(ctx, counters));
    comps = ctx->host_pinned[kCntComponents];
    status = RST_E_DISCONNECTED;
  }
  RST_TRY(mark(ctx, stats, 2));
  if (stats) {
    RST_HIP(hipEventSynchronize(ctx->ev[2]));
    static const int gaps[2] = {RST_STAGE_BFS, RST_STAGE_BFS};
    fill_stage_times(ctx, stats, gaps, 3);
    stats->bfs_levels = levels;
    stats->components = comps;
    stats->method_used = RST_BFS;
  }
  return status;
}

rst_status rst_components(rst_ctx *ctx, const rst_csr *g, int32_t *label,
                          int64_t *num_components) {
  if (!ctx || !label) return RST_E_INVAL;
  RST_TRY(check_csr(g));
  RST_HIP(hipSetDevice(ctx->device));
  const int64_t chunk_cap = (int64_t)hook_chunk_capacity(ctx, g->nnz);
  RST_TRY(ws_reserve(ctx, ws_bytes(64, 4) + 2 * ws_bytes(g->n, 4) + hook_ws_bytes(ctx, g)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  RST_TRY(enqueue_fill(ctx, counters, 32, 0));
  RST_TRY(run_validation(ctx, g, counters));
  ForestBufs f;
  f.counters = counters;
  f.cc = label;
  f.tu = ws_take<int32_t>(ctx, g->n);
  f.tv = ws_take<int32_t>(ctx, g->n);
  int64_t *chunks = ws_take<int64_t>(ctx, chunk_cap);
  int2 *cross = ws_take<int2>(ctx, hook_cross_capacity(g->nnz));
  int32_t *tile_cross = ws_take<int32_t>(ctx, hook_tile_words(g->n));
  bool global_hook = false;
  RST_TRY(choose_hook(ctx, g, f.vmask, f.counters, &global_hook));
  RST_TRY(enqueue_hook(ctx, g, f, global_hook, chunks, chunk_cap, cross, tile_cross));
  RST_TRY(enqueue_compress(ctx, g->n, label, nullptr, nullptr));
  RST_TRY(enqueue_count_roots(ctx, g->n, label, counters));
  RST_TRY(read_counters(ctx, counters));
  if (num_components) *num_components = ctx->host_pinned[kCntComponents];
  return RST_OK;
}

rst_status rst_verify(rst_ctx *ctx, const rst_csr *g, int32_t root, const int32_t *parent,
                      int64_t *num_failures, int64_t *first_bad) {
  if (!ctx || !parent || !num_failures) return RST_E_INVAL;
  RST_TRY(check_csr(g));
  if (root < 0 || root >= g->n) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  const int64_t n = g->n;
  const int64_t chunk_cap = (int64_t)hook_chunk_capacity(ctx, g->nnz);
  RST_TRY(ws_reserve(ctx, ws_bytes(64, 4) + 5 * ws_bytes(n, 4) + hook_ws_bytes(ctx, g)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  int32_t *vc = counters + 40;
  RST_TRY(enqueue_fill(ctx, counters, 32, 0));
  RST_TRY(enqueue_fill(ctx, vc, 1, 0));
  RST_TRY(enqueue_fill(ctx, vc + 1, 1, 0x7fffffff));
  RST_TRY(run_validation(ctx, g, counters));
  // component labels of the graph (min ids) by the library's own hooking
  ForestBufs f;
  f.counters = counters;
  f.cc = ws_take<int32_t>(ctx, n);
  f.tu = ws_take<int32_t>(ctx, n);
  f.tv = ws_take<int32_t>(ctx, n);
  int64_t *chunks = ws_take<int64_t>(ctx, chunk_cap);
  int2 *cross = ws_take<int2>(ctx, hook_cross_capacity(g->nnz));
  int32_t *tile_cross = ws_take<int32_t>(ctx, hook_tile_words(n));
  bool global_hook = false;
  RST_TRY(choose_hook(ctx, g, f.vmask, f.counters, &global_hook));
  RST_TRY(enqueue_hook(ctx, g, f, global_hook, chunks, chunk_cap, cross, tile_cross));
  RST_TRY(enqueue_compress(ctx, n, f.cc, nullptr, nullptr));
  int32_t *anc0 = ws_take<int32_t>(ctx, n);
  int32_t *anc1 = ws_take<int32_t>(ctx, n);
  RST_TRY(enqueue_verify(ctx, g, root, f.cc, parent, anc0, anc1, vc));
  RST_HIP(hipMemcpyAsync(ctx->host_pinned + 40, vc, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                         ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  *num_failures = ctx->host_pinned[40];
  if (first_bad) *first_bad = ctx->host_pinned[40] ? ctx->host_pinned[41] : -1;
  return RST_OK;
}

rst_status rst_spanning_forest(rst_ctx *ctx, const rst_csr *g, int32_t *label, int32_t *tu,
                               int32_t *tv, int64_t *num_edges) {
  if (!ctx || !label || !tu || !tv) return RST_E_INVAL;
  RST_TRY(check_csr(g));
  RST_HIP(hipSetDevice(ctx->device));
  const int64_t chunk_cap = (int64_t)hook_chunk_capacity(ctx, g->nnz);
  RST_TRY(ws_reserve(ctx, ws_bytes(64, 4) + hook_ws_bytes(ctx, g)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  RST_TRY(enqueue_fill(ctx, counters, 32, 0));
  RST_TRY(run_validation(ctx, g, counters));
  ForestBufs f;
  f.counters = counters;
  f.cc = label;
  f.tu = tu;
  f.tv = tv;
  int64_t *chunks = ws_take<int64_t>(ctx, chunk_cap);
  int2 *cross = ws_take<int2>(ctx, hook_cross_capacity(g->nnz));
  int32_t *tile_cross = ws_take<int32_t>(ctx, hook_tile_words(g->n));
  bool global_hook = false;
  RST_TRY(choose_hook(ctx, g, f.vmask, f.counters, &global_hook));
  RST_TRY(enqueue_hook(ctx, g, f, global_hook, chunks, chunk_cap, cross, tile_cross));
  RST_TRY(enqueue_compress(ctx, g->n, label, nullptr, nullptr));
  RST_TRY(enqueue_count_roots(ctx, g->n, label, counters));
  RST_TRY(read_counters(ctx, counters));
  if (num_edges) *num_edges = g->n - ctx->host_pinned[kCntComponents];
  return RST_OK;
}

rst_status rst_bfs(rst_ctx *ctx, const rst_csr *g, int32_t root, int32_t *level, int32_t *parent,
                   rst_stats *stats) {
  if (!ctx || !level || !parent) return RST_E_INVAL;
  RST_TRY(check_csr(g));
  if (root < 0 || root >= g->n) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  if (stats) std::memset(stats, 0, sizeof(*stats));
  RST_TRY(ws_reserve(ctx, ws_bytes(64, 4) + bfs_ws_bytes(ctx, g)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  int32_t *rootbuf = counters + 32;
  RST_TRY(enqueue_reset_counters(ctx, counters, root));
  RST_TRY(run_validation(ctx, g, counters));
  BfsBufs b;
  RST_TRY(take_bfs_bufs(ctx, g, b));
  RST_TRY(mark(ctx, stats, 0));
  RST_TRY(bfs_reset(ctx, g->n, level, parent, b));
  RST_TRY(bfs_seed_roots(ctx, g, rootbuf, 1, level, parent, b, counters));
  int64_t levels = 0;
  RST_TRY(bfs_run_levels(ctx, g, level, parent, b, counters, &levels));
  RST_TRY(mark(ctx, stats, 1));
  if (stats) {
    RST_HIP(hipEventSynchronize(ctx->ev[1]));
    static const int gaps[1] = {RST_STAGE_BFS};
    fill_stage_times(ctx, stats, gaps, 2);
    stats->bfs_levels = levels;
    stats->method_used = RST_BFS;
  }
  return RST_OK;
}

rst_status rst_root_forest(rst_ctx *ctx, int64_t n, int64_t t, const int32_t *eu,
                           const int32_t *ev, const int32_t *roots, int32_t nroots,
                           int32_t *parent) {
  if (!ctx || !parent || n < 1 || t < 0 || t > n - 1 || nroots < 0) return RST_E_INVAL;
  if (t > 0 && (!eu || !ev)) return RST_E_INVAL;
  if (nroots > 0 && !roots) return RST_E_INVAL;
  if (n >= ((int64_t)1 << 30)) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  const int64_t lists = (t < n / 2 ? t : n / 2) + 1;
  const GlistPlan plan = glist_plan(2 * t, lists, ctx->opt.rank_stride);
  RST_TRY(ws_reserve(ctx, ws_bytes(64, 4) + 5 * ws_bytes(n, 4) + 2 * ws_bytes(2 * t + 2, 4) +
                              ws_bytes(2 * t + 2, 8) + rank_ws_bytes(2 * t) +
                              glist_ws_bytes(plan)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  int32_t *cc = ws_take<int32_t>(ctx, n);
  int32_t *comp_root = ws_take<int32_t>(ctx, n);
  int32_t *head = ws_take<int32_t>(ctx, n);
  int32_t *endsucc = ws_take<int32_t>(ctx, n);
  int32_t *next = ws_take<int32_t>(ctx, 2 * t + 2);
  uint64_t *rank = ws_take<uint64_t>(ctx, 2 * t + 2);
  int32_t *xid = ws_take<int32_t>(ctx, 2 * t + 2);
  RankBufs rb = take_rank_bufs(ctx, 2 * t);
  GlistBufs gl;
  glist_take(ctx, plan, gl);
  RST_TRY(enqueue_fill(ctx, counters, 32, 0));
  RST_TRY(enqueue_hook_coo(ctx, n, t, eu, ev, cc, counters));
  RST_TRY(enqueue_compress(ctx, n, cc, comp_root, head));
  RST_TRY(read_counters(ctx, counters));
  if (ctx->host_pinned[kCntRangeErr]) return RST_E_INVAL;
  RST_TRY(enqueue_mark_roots(ctx, roots, nroots, n, cc, comp_root, parent, counters));
  RST_TRY(enqueue_link(ctx, t, eu, ev, head, next));
  SlotArcs arcs{eu, ev, next, head, cc, comp_root, n, endsucc};
  RST_TRY(enqueue_rank_tiled(ctx, 2 * t, rank, xid, rb, counters, &arcs, false));
  RST_TRY(enqueue_expand_parent(ctx, t, n, eu, ev, rank, xid, rb.tile_base, rb.crank, cc,
                                comp_root, parent, counters));
  RST_TRY(read_counters(ctx, counters));
  if (ctx->host_pinned[kCntRankOverflow]) {
    // contracted list too long for one workgroup: the sparse ruling set over
    // the tour (endsucc was filled by the per-tile pass)
    int32_t *w1 = reinterpret_cast<int32_t *>(rank);
    RST_TRY(enqueue_fill(ctx, counters + kCntRankOverflow, 1, 0));
    RST_TRY(enqueue_glist_from_slots(ctx, t, n, eu, ev, next, endsucc, head, w1, gl, counters));
    RST_TRY(enqueue_glist_rank(ctx, w1, false, gl, counters));
    RST_TRY(enqueue_glist_parent(ctx, t, n, eu, ev, w1, gl, cc, comp_root, parent, counters,
                                 nullptr));
    RST_TRY(read_counters(ctx, counters));
    if (ctx->host_pinned[kCntGOverflow]) {
      RST_TRY(glist_wyllie_parent(ctx, t, n, eu, ev, next, endsucc, rank, cc, comp_root, parent,
                                  counters));
      RST_TRY(read_counters(ctx, counters));
    }
  }
  if (ctx->host_pinned[kCntRangeErr] || ctx->host_pinned[kCntRootErr]) return RST_E_INVAL;
  return RST_OK;
}

rst_status rst_list_rank(rst_ctx *ctx, int64_t A, const int32_t *succ, int32_t *dist) {
  if (!ctx || A < 0 || (A > 0 && (!succ || !dist))) return RST_E_INVAL;
  if (A >= ((int64_t)1 << 31)) return RST_E_INVAL;
  if (A == 0) return RST_OK;
  RST_HIP(hipSetDevice(ctx->device));
  const GlistPlan plan = glist_plan(A, A, ctx->opt.rank_stride);
  RST_TRY(ws_reserve(ctx, ws_bytes(64, 4) + ws_bytes(A, 8) + ws_bytes(A, 4) + rank_ws_bytes(A) +
                              glist_ws_bytes(plan)));
  int32_t *counters = ws_take<int32_t>(ctx, 64);
  uint64_t *rank = ws_take<uint64_t>(ctx, A);
  int32_t *xid = ws_take<int32_t>(ctx, A);
  RankBufs rb = take_rank_bufs(ctx, A);
  GlistBufs gl;
  glist_take(ctx, plan, gl);
  RST_TRY(enqueue_fill(ctx, counters, 32, 0));
  RST_TRY(enqueue_rank_init(ctx, A, succ, rank));
  RST_TRY(enqueue_rank_tiled(ctx, A, rank, xid, rb, counters, nullptr, true));
  RST_TRY(read_counters(ctx, counters));
  if (ctx->host_pinned[kCntRankOverflow]) {
    // contracted list too long for one workgroup: the sparse ruling set over
    // the input lists (level-1 words in rank, has-predecessor bytes in xid)
    int32_t *w1 = reinterpret_cast<int32_t *>(rank);
    RST_TRY(enqueue_fill(ctx, counters + kCntRankOverflow, 1, 0));
    RST_TRY(enqueue_glist_from_succ(ctx, A, succ, w1, reinterpret_cast<uint8_t *>(xid), gl,
                                    counters));
    RST_TRY(enqueue_glist_rank(ctx, w1, false, gl, counters));
    RST_TRY(enqueue_glist_dist(ctx, A, w1, gl, dist, counters));
    RST_TRY(read_counters(ctx, counters));
    if (ctx->host_pinned[kCntGOverflow]) {
      // more lists than the sparse ruling set holds: Wyllie rounds over all nodes
      RST_TRY(enqueue_rank_init(ctx, A, succ, rank));
      RST_TRY(enqueue_rank_rounds(ctx, A, rank, rank_rounds_for(A), nullptr, nullptr));
      RST_TRY(enqueue_rank_extract(ctx, A, rank, dist));
    }
    RST_HIP(hipStreamSynchronize(ctx->stream));
    return RST_OK;
  }
  RST_TRY(enqueue_rank_extract(ctx, A, rank, dist));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  return RST_OK;
}

rst_status rst_spanning_forest_batch(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                     const uint8_t *method, int32_t *parent, uint8_t *method_out,
                                     rst_stats *stats) {
  if (!ctx || !parent || !b || b->num_graphs < 1 || !b->vtx_off || !b->arc_off || !b->roots)
    return RST_E_INVAL;
  RST_TRY(check_csr(g));
  if (b->num_graphs > g->n) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  if (stats) std::memset(stats, 0, sizeof(*stats));
  TimingScope timing(ctx, stats != nullptr);
  const int32_t G = b->num_graphs;
  const int64_t n = g->n;
  RST_TRY(ws_reserve(ctx, ws_bytes(64, 4) + gconn_ws_bytes(ctx, g) + bfs_ws_bytes(ctx, g) +
                              ws_bytes(n, 4) + 2 * ws_bytes(n, 1) + ws_bytes(G, 1) + ws_bytes(G, 4) +
                              (method ? 0 : selector_scratch_bytes(ctx, g, G))));
  BatchWork bw;
  bw.counters = ws_take<int32_t>(ctx, 64);
  bw.m = ws_take<uint8_t>(ctx, G);
  bw.vmask = ws_take<uint8_t>(ctx, n);
  bw.gsel = ws_take<uint8_t>(ctx, n);
  bw.level = ws_take<int32_t>(ctx, n);
  RST_TRY(take_bfs_bufs(ctx, g, bw.bb));
  int32_t *giants = ws_take<int32_t>(ctx, G);
  bw.w = take_gconn_work(ctx, g, bw.counters, nullptr, bw.vmask);
  // the global sweep seeks a dominant tree in every packed graph; with the
  // hooking variant left to the library, each graph gets its own (tile pass
  // where its ids carry locality, global sweep where they do not)
  bw.w.f.vtx_off = b->vtx_off;
  bw.w.f.num_graphs = G;
  bw.w.f.giants = giants;
  if (ctx->opt.hook_mode == 0 && G > 1 && g->nnz < ((int64_t)1 << 31)) bw.w.f.gsel = bw.gsel;
  bw.sel_scratch = ctx->ws.used;   // the selector's scratch follows (method == NULL)

  const bool graph_path = ctx->opt.graphs && !stats && !ctx->opt.validate;
  GraphKey key;
  std::memset(&key, 0, sizeof key);
  key.offsets = g->offsets; key.cols = g->cols; key.parent = parent;
  key.ws_base = ctx->ws.base; key.ws_cap = (int64_t)ctx->ws.cap;
  key.n = g->n; key.nnz = g->nnz; key.offset_bytes = g->offset_bytes;
  key.opt = ctx->opt;
  key.vtx_off = b->vtx_off; key.arc_off = b->arc_off; key.roots = b->roots;
  key.method = method; key.method_out = method_out;
  key.selector = method ? nullptr : selector_weights(ctx);
  key.num_graphs = G; key.batch = 1;

  if (!graph_path || !ctx->graph || !(ctx->graph->key == key)) {
    // eager: the hooking variant from the locality probe, the ranking from the
    // hooking counters, BFS levels until the frontier is empty
    bool sparse = false, global_hook = false;
    const rst_status st = run_batch_eager(ctx, g, b, method, parent, method_out, stats, bw,
                                          &sparse, &global_hook);
    if (graph_path && st == RST_OK) {
      graph_forget(ctx);
      ctx->graph->key = key;
      ctx->graph->sparse = sparse;
      ctx->graph->global_hook = global_hook;
    }
    return st;
  }
  // replay: the whole device part without a host round trip, then one
  // synchronisation and the rare continuations
  bw.w.sparse = ctx->graph->sparse;
  bw.w.global_hook = ctx->graph->global_hook;
  bw.w.settled = G == 1;   // as enqueue_gconn_forest decides (a replay runs no host code)
  RST_TRY(run_graph(ctx, key, [&]() -> rst_status {
    return enqueue_batch_device(ctx, g, b, method, parent, method_out, bw, kBatchBfsSteps);
  }));
  return finish_batch(ctx, g, b, parent, bw, nullptr);
}

rst_status rst_tree_depth(rst_ctx *ctx, int64_t n, const int32_t *parent, int32_t *depth,
                          int64_t *max_depth) {
  if (!ctx || !parent || !depth || n < 1) return RST_E_INVAL;
  if (n >= ((int64_t)1 << 30)) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  return run_tree_depth(ctx, n, parent, depth, max_depth);
}

const char *rst_status_string(rst_status s) {
  switch (s) {
    case RST_OK: return "ok";
    case RST_E_INVAL: return "invalid argument";
    case RST_E_NOMEM: return "out of device memory";
    case RST_E_DEVICE: return "HIP runtime error";
    case RST_E_DISCONNECTED: return "graph is disconnected (spanning forest returned)";
    case RST_E_RANGE: return "offset or neighbour id out of range";
    case RST_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

}  // extern "C"
