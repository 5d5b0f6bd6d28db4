/*
 * rst.h -- C ABI of librst, rooted spanning trees on AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. I of "Beyond BFS: A Comparative Study of Rooted Spanning Tree
 * Algorithms on GPUs", arXiv 2603.11645): given an undirected connected graph
 * G=(V,E) and a root r, return a parent array P with P[r] = r and exactly one
 * parent for every other vertex, each {v, P[v]} an edge of G.
 *
 * Two methods are provided:
 *   RST_GCONN_EULER  connectivity by hooking + pointer jumping that records the
 *                    edge behind every union (Sec. III-B), then Euler-tour
 *                    rooting of the spanning forest (Sec. III-D);
 *   RST_BFS          level-synchronous breadth-first search (Sec. III-A);
 *   RST_PR_RST       Path-Reversal RST (Sec. III-C): a rooted forest kept
 *                    through hooking rounds that alternate max and min
 *                    representatives, each graft re-rooting the grafted tree
 *                    by reversing the path marked through its vertices'
 *                    ancestors at power-of-two distances.
 *
 * Conventions shared by every call:
 *   - Every array argument is a DEVICE pointer unless its comment says host.
 *     The caller owns and allocates all input and output buffers; the library
 *     only reads inputs and writes outputs and never frees them.
 *   - Vertex ids are int32; 0 <= id < n.  Offsets are int32 or int64 as given by
 *     rst_csr.offset_bytes.  The CSR must be symmetric (both directions of every
 *     undirected edge stored); self-loops and duplicate arcs are tolerated.
 *   - Calls are synchronous: work is enqueued on the context's HIP stream and the
 *     call returns after that work has completed.  One context per host thread.
 *   - Every call returns an rst_status; no call aborts and no C++ exception
 *     crosses the ABI.  On an error other than RST_E_DISCONNECTED the contents of
 *     output buffers are unspecified.
 *   - Device scratch memory is owned by the context, grown on demand with
 *     hipMalloc, and released by rst_destroy.
 */
#ifndef RST_H
#define RST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rst_ctx rst_ctx;

typedef enum {
  RST_OK = 0,
  RST_E_INVAL = -1,        /* null pointer, n < 1, root out of range, bad offset width,
                              nnz too large for 4-byte offsets, ...                     */
  RST_E_NOMEM = -2,        /* device scratch allocation failed                          */
  RST_E_DEVICE = -3,       /* a HIP runtime call failed                                 */
  RST_E_DISCONNECTED = -4, /* input has more than one component; the output is still a
                              valid rooted spanning forest (see rst_spanning_tree)       */
  RST_E_RANGE = -5,        /* validation found an offset or neighbour id out of range   */
  RST_E_UNSUPPORTED = -6   /* request not supported by this build / device              */
} rst_status;

typedef enum { RST_GCONN_EULER = 0, RST_BFS = 1, RST_AUTO = 2, RST_PR_RST = 3 } rst_method;

/* Symmetric CSR of an undirected graph (Sec. I). */
typedef struct {
  int64_t n;             /* vertices, >= 1                                          */
  int64_t nnz;           /* stored arcs = offsets[n]                                */
  int32_t offset_bytes;  /* 4 (int32 offsets, nnz < 2^31) or 8 (int64 offsets)     */
  const void *offsets;   /* device [n+1], non-decreasing, offsets[0] = 0            */
  const int32_t *cols;   /* device [nnz], neighbour ids                             */
} rst_csr;

/* Several graphs packed into one CSR with global vertex ids: graph g owns
 * vertices [vtx_off[g], vtx_off[g+1]) and arcs [arc_off[g], arc_off[g+1]). */
typedef struct {
  int32_t num_graphs;      /* G >= 1                                              */
  const int64_t *vtx_off;  /* device [G+1]                                        */
  const int64_t *arc_off;  /* device [G+1]                                        */
  const int32_t *roots;    /* device [G], global id of each graph's root          */
} rst_batch;

/* Stage indices of rst_stats.ms_stage. */
enum {
  RST_STAGE_HOOK = 0,      /* hooking sweep (spanning-edge recording)           */
  RST_STAGE_COMPRESS = 1,  /* pointer jumping to min-id labels                  */
  RST_STAGE_ARCS = 2,      /* root marking + twin arcs and per-vertex arc lists */
  RST_STAGE_SUCC = 3,      /* Euler successor + cycle breaking                  */
  RST_STAGE_RANK = 4,      /* list ranking (all rounds)                         */
  RST_STAGE_PARENT = 5,    /* parents from tour order                           */
  RST_STAGE_BFS = 6,       /* breadth-first search (all levels)                 */
  RST_STAGE_SELECT = 7     /* selector features + inference (batch calls)       */
};

/* Host struct filled by calls that take an rst_stats* (nullable).  Timings are
 * HIP-event times on the context stream; they are only collected when the
 * pointer is non-NULL (events add a little overhead). */
typedef struct {
  float ms_total;
  float ms_stage[8];
  float ms_kernel[12];    /* single kernels, see RST_KERNEL_*                  */
  int64_t hook_rounds;    /* levels of the binary tree over vertex tiles + 1   */
  int64_t rank_rounds;    /* pointer-jumping rounds on the contracted list     */
  int64_t rank_exits;     /* length of the contracted list (segment exits)     */
  int64_t cross_edges;    /* edges left to the cross-tile phase of hooking     */
  int64_t bfs_levels;     /* deepest BFS level reached (eccentricity of root)  */
  int64_t components;     /* connected components found                        */
  int32_t method_used;    /* rst_method actually run (batch: -1 if mixed)      */
  int32_t paths;          /* RST_PATH_* bits: which variant of a stage ran     */
} rst_stats;

/* Bits of rst_stats.paths.  Stages first try a one-workgroup variant and fall
 * back to a multi-workgroup one when their data do not fit it. */
enum {
  RST_PATH_CROSS_GLOBAL = 1,  /* cross-tile merge ran in global memory (the     *
                               * kept cross edges did not fit one workgroup)    */
  RST_PATH_RANK_GLOBAL = 2,   /* last resort: every arc ranked by multi-        *
                               * workgroup pointer-jumping rounds (more lists   *
                               * than the sparse ruling set holds)              */
  RST_PATH_CROSS_GROUPS = 4,  /* kept cross edges too many for the one-workgroup *
                               * merge of all levels: merged per group of tiles *
                               * and then the top levels (graphs of more than   *
                               * 8 tiles of 8192 vertices only)                 */
  RST_PATH_RANK_SPARSE = 8,   /* the tour was ranked by the sparse ruling set in *
                               * global memory (ids without locality), not per  *
                               * arc tile                                        */
  RST_PATH_HOOK_GLOBAL = 16,  /* hooking swept the CSR in global memory (ids     *
                               * without locality), no vertex tiles              */
  RST_PATH_HOOK_GIANT = 32    /* ... after sampling each vertex's first arcs,    *
                               * with the vertices of the dominant tree skipped  */
};

/* Indices of rst_stats.ms_kernel (HIP-event time of one launch each). */
enum {
  RST_KERNEL_HOOK_TILE = 0,   /* LDS union-find over vertex tiles               */
  RST_KERNEL_CROSS = 1,       /* all cross-tile hooking levels together         */
  RST_KERNEL_RANK_TILE = 2,   /* LDS ruling-set ranking over arc tiles (+succ)  */
  RST_KERNEL_LINK = 3,        /* per-vertex out-arc lists                       */
  RST_KERNEL_RANK_WALK = 4,   /* sparse ruling set in global memory: the walks  *
                               * of the first level (tours without id locality) */
  RST_KERNEL_LATE_HOOKS = 5,  /* global-memory hooking of cross edges that the  *
                               * LDS merges did not take, and heavy vertices     */
  RST_KERNEL_SETTLE = 6,      /* one-root pass: roots, end-of-list successors    */
  RST_KERNEL_PARENT = 7,      /* parent rule from the ranks (either ranking)     */
  RST_KERNEL_RANK_WORDS = 8,  /* sparse ruling set: successors of every arc from *
                               * the forest slots, list heads                    */
  RST_KERNEL_HOOK_SAMPLE = 9, /* global hooking: initialisation, sampled arcs,   *
                               * dominant root (three launches together)         */
  RST_KERNEL_HOOK_GLOBAL = 10 /* global hooking: the sweep over the CSR          */
};

/* Tunables and switches for rst_set_option. */
typedef enum {
  RST_OPT_VALIDATE = 0,        /* 1: check offsets/neighbour ids before running (O(nnz)) */
  RST_OPT_BFS_LEVELS_PER_SYNC = 1, /* BFS levels launched between host checks (>= 1)   */
  RST_OPT_BFS_GRID = 2,        /* blocks per BFS level launch (0 = automatic)          */
  RST_OPT_RANK_ELEMS_PER_THREAD = 3, /* words per thread of the multi-workgroup list-
                                      * ranking rounds (1, 2, 4, 8)                 */
  RST_OPT_HEAVY_DEGREE = 4,    /* hooking: degree above which a vertex's arcs are cut
                                * into chunks hooked by many workgroups (32 .. 2^24;
                                * values above 1023 act as 1023: the tile pass
                                * takes no vertex of larger degree)                */
  RST_OPT_SWEEP_BLOCK = 5,     /* threads per workgroup of the per-vertex and per-slot
                                * sweeps (64, 128, 256, 512, 1024)                 */
  RST_OPT_BFS_HEAVY_DEGREE = 6, /* BFS: degree above which a frontier vertex's arcs are
                                 * expanded by many workgroups (32 .. 2^24)         */
  RST_OPT_GRAPHS = 7,          /* 1 (default): rst_spanning_tree by GConn+Euler without
                                * stats or validation runs eagerly on the first call
                                * with given graph pointers, sizes, root, parent
                                * buffer and settings, captures its device work as a
                                * HIP graph on the second and replays it while they
                                * stay the same; 0: launch eagerly                 */
  RST_OPT_RANK_STRIDE = 8,     /* sparse ruling set (tours without id locality):
                                * every k-th arc starts a ruler, k in 4, 8, 16, 32,
                                * 64; 0 (default): 16, or 32 above 2^24 arcs      */
  RST_OPT_HOOK_MODE = 9,       /* hooking of GConn+Euler and rst_components: 0
                                * (default) chooses by sampling arcs: when most
                                * leave their source's 8192-id tile the global
                                * sweep runs, else the tile pass; 1: tile pass;
                                * 2: global sweep (needs nnz < 2^31, else tiles) */
  RST_OPT_HOOK_SAMPLE = 10     /* global sweep: arcs per vertex hooked before the
                                * dominant tree is sought, 0 .. 4; -1 (default):
                                * 2 when nnz >= 6 n, else 0                       */
} rst_option;
#define RST_NUM_OPTIONS 11

/* Create a context on HIP device `device` bound to `hip_stream` (a hipStream_t,
 * NULL = the default stream).  *out receives the context.  Errors: RST_E_INVAL
 * (out == NULL or bad device), RST_E_DEVICE. */
rst_status rst_create(rst_ctx **out, int device, void *hip_stream);

/* Release the context and its scratch memory.  NULL is ignored. */
void rst_destroy(rst_ctx *ctx);

/* Rebind the context to another stream of the same device. */
rst_status rst_set_stream(rst_ctx *ctx, void *hip_stream);

/* Set a tunable (see rst_option).  RST_E_INVAL for an unknown option or a value
 * out of range.  Every value gives the same results; only the speed changes. */
rst_status rst_set_option(rst_ctx *ctx, rst_option opt, int64_t value);

/* Current value of a tunable into *value (host).  RST_E_INVAL for an unknown
 * option or NULL pointers. */
rst_status rst_get_option(const rst_ctx *ctx, rst_option opt, int64_t *value);

/* Rooted spanning tree of the graph (Sec. I) by `method` (RST_AUTO runs the
 * selector on this one graph; RST_PR_RST reports its hooking iterations in
 * stats->hook_rounds).  parent: device int32 [n], written completely.
 * If the graph is disconnected the call returns RST_E_DISCONNECTED and parent
 * is a rooted spanning forest: root's component is rooted at root, every other
 * component at its minimum vertex id.  stats may be NULL. */
rst_status rst_spanning_tree(rst_ctx *ctx, const rst_csr *g, int32_t root, rst_method method,
                             int32_t *parent, rst_stats *stats);

/* Connected components by hooking + pointer jumping (Sec. III-B).  label: device
 * int32 [n] receives the minimum vertex id of each vertex's component.
 * num_components: host, nullable. */
rst_status rst_components(rst_ctx *ctx, const rst_csr *g, int32_t *label,
                          int64_t *num_components);

/* Component labels as rst_components, allocating nothing: for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Hooking always runs the global
 * sweep (RST_OPT_HOOK_MODE is ignored).  Its scratch is one fixed 128 MiB
 * device array per GPU, held from the first context on that GPU until the
 * process ends, so n <= 16,777,184 and nnz < 2^31 are required (else
 * RST_E_INVAL, nothing is run).  Every call on a GPU uses that GPU's array and
 * clears what must start at zero: calls that overlap on one GPU race.
 * label: device int32 [n]; num_components: host, nullable.  Synchronous. */
rst_status rst_components_noalloc(rst_ctx *ctx, const rst_csr *g, int32_t *label,
                                  int64_t *num_components);

/* The connectivity stage alone (Sec. III-B with the spanning-edge marking of
 * Sec. I): label as in rst_components, and for every vertex x that stopped being
 * a component root, the graph edge (tu[x], tv[x]) whose hook made it a non-root;
 * tu[x] = tv[x] = -1 for the n - t vertices that stayed roots.  tu, tv: device
 * int32 [n].  num_edges: host, nullable, receives t = n - components. */
rst_status rst_spanning_forest(rst_ctx *ctx, const rst_csr *g, int32_t *label, int32_t *tu,
                               int32_t *tv, int64_t *num_edges);

/* Level-synchronous BFS from root (Sec. III-A).  level: device int32 [n], hop
 * distance or -1 if unreachable; parent: device int32 [n], a neighbour one level
 * closer to root (parent[root] = root), -1 if unreachable.  Returns RST_OK even
 * if some vertices are unreachable.  stats may be NULL. */
rst_status rst_bfs(rst_ctx *ctx, const rst_csr *g, int32_t root, int32_t *level,
                   int32_t *parent, rst_stats *stats);

/* The Euler-tour rooting stage alone (Sec. III-D) for a forest given as t
 * undirected edges (eu[k], ev[k]) over n vertices (device int32 [t] each).
 * roots: device int32 [nroots], at most one per tree; a tree without a listed
 * root is rooted at its minimum vertex id.  parent: device int32 [n].  The
 * result is unique for a given forest and roots.  RST_E_INVAL if two roots share
 * a tree or the edges are out of range; a non-forest input (a cycle) gives an
 * unspecified parent array. */
rst_status rst_root_forest(rst_ctx *ctx, int64_t n, int64_t t, const int32_t *eu,
                           const int32_t *ev, const int32_t *roots, int32_t nroots,
                           int32_t *parent);

/* List ranking (Sec. III-D): succ is a device int32 [A] array describing
 * disjoint simple lists (succ[e] = next node or -1 at a tail).  dist: device
 * int32 [A] receives the number of nodes after e in its list (0 at the tail).
 * Cycles give unspecified output. */
rst_status rst_list_rank(rst_ctx *ctx, int64_t A, const int32_t *succ, int32_t *dist);

/* Depth of every vertex of a rooted forest (the tree-depth comparison of
 * Sec. IV-B, Fig. 2), computed from its Euler tour (Sec. III-D): arcs weigh
 * +1 going down and -1 going up, and the depth of v is the weighted position
 * of the arc into v, found by weighted list ranking.  parent: device int32
 * [n], P[r] = r at roots (an entry outside [0, n) is taken as a root); depth:
 * device int32 [n] receives the number of tree edges from each vertex to its
 * root; max_depth: host, nullable, receives the largest.  A parent array with
 * a cycle gives unspecified depths for the vertices on or below it. */
rst_status rst_tree_depth(rst_ctx *ctx, int64_t n, const int32_t *parent, int32_t *depth,
                          int64_t *max_depth);

/* Biconnected components of a connected graph from a rooted spanning tree of
 * it: the downstream use of an RST that Sec. I and the opening of Sec. IV name
 * (Tarjan and Vishkin's method).  The tree's preorder numbers and subtree
 * sizes come from its Euler tour (Sec. III-D), weighted 1 on down arcs and 0
 * on up arcs and ranked like rst_tree_depth's; tree edges are joined when a
 * subtree reaches past its parent's subtree or a non-tree edge links them,
 * and the connected components of those joins (hooking + pointer jumping,
 * Sec. III-B) are the biconnected components.
 * g: the graph (nnz < 2^31); parent: device int32 [n], a rooted spanning
 * tree of g with one root (P[r] = r; e.g. from rst_spanning_tree; check it
 * with rst_verify: any other array gives unspecified labels, never an access
 * outside the buffers).  arc_label: device int32 [nnz] receives for every arc
 * the label of its component -- the smallest vertex v whose tree edge
 * {P[v], v} lies in it -- and -1 for self-loops; articulation: device uint8
 * [n], nullable, receives 1 for every vertex whose arcs lie in two or more
 * components; num_components: host, nullable.  Errors: RST_E_INVAL,
 * RST_E_DISCONNECTED (parent has more than one root), RST_E_RANGE (its tour
 * gives preorder numbers outside [0, n): not a tree).  Synchronous. */
rst_status rst_biconnected(rst_ctx *ctx, const rst_csr *g, const int32_t *parent,
                           int32_t *arc_label, uint8_t *articulation, int64_t *num_components);

/* Rooted spanning forest of G packed graphs in one pass: graph g is rooted at
 * roots[g].  method: device uint8 [G] per graph (0 = GConn+Euler, nonzero =
 * BFS), or NULL to let the loaded selector choose (GConn+Euler if none is
 * loaded).  parent: device int32 [total n]; a graph that is itself
 * disconnected gets its other components rooted at their minimum ids.
 * method_out: device uint8 [G], nullable, receives the method used per graph.
 * The number of kernel launches does not depend on G.  RST_E_INVAL if the
 * offset tables disagree with the CSR or a root lies outside its graph; with
 * RST_OPT_VALIDATE, RST_E_RANGE if an arc's neighbour lies outside the arc's
 * graph.
 * stats may be NULL. */
rst_status rst_spanning_forest_batch(rst_ctx *ctx, const rst_csr *g, const rst_batch *b,
                                     const uint8_t *method, int32_t *parent,
                                     uint8_t *method_out, rst_stats *stats);

/* ---- learned BFS / GConn+Euler selector (per graph of a batch) ------------
 * Features of graph g, feat[g*8 + k]: log n, log(1 + m), mean degree,
 * log(1 + degree variance), log(1 + max degree), and for probes s = 0, 1, 2
 * log2(1 + d), d = the depth a BFS from the source reaches before it stops:
 * min(eccentricity of the source, 64, the first radius whose ball -- the
 * vertices within that many hops -- holds at least 1024 vertices); the source
 * is vtx_off[g] + (the (3g + s + 1)-th output of the splitmix64 generator seeded
 * with 0) mod n_g (splitmix64: Steele, Lea, Flood 2014; state += 0x9E3779B97F4A7C15,
 * then the finaliser).  Degree moments use arcs of the
 * CSR; m counts each undirected edge once (arcs / 2).
 * Network: 8 -> 64 -> 64 -> 2 fully connected, ReLU, fp32, applied to z-scored
 * features (x - mean) / max(std, 1e-6).  Output 0 scores GConn+Euler, output 1
 * scores BFS; BFS is chosen only when its score is strictly larger and every
 * feature and score is finite.
 * Parameter vector (4866 floats, row-major): W1[64][8], b1[64], W2[64][64],
 * b2[64], W3[2][64], b3[2].  Normalisation vector: mean[8], std[8].
 * Selector blob (host bytes, little endian): "RSTSEL01" (8 bytes), int32 8,
 * int32 64, then 16 floats of normalisation and the 4866 parameters; total
 * 16 + 4 * 4882 = 19544 bytes. */

/* Features of every graph of a packed batch.  feat: device float [G*8]. */
rst_status rst_features(rst_ctx *ctx, const rst_csr *g, const rst_batch *b, float *feat);

/* Column mean and standard deviation of X (device float [B*8]) into norm
 * (device float [16]: mean[8] then std[8]), accumulated in double. */
rst_status rst_feature_stats(rst_ctx *ctx, const float *X, int64_t B, float *norm);

/* Forward pass for B feature rows X (device float [B*8]).  logits: device
 * float [B*2] (nullable); choice: device uint8 [B] (nullable) receives 1 for
 * BFS, 0 for GConn+Euler.  norm/params: device, layouts above. */
rst_status rst_mlp_forward(rst_ctx *ctx, const float *norm, const float *params, const float *X,
                           int64_t B, float *logits, uint8_t *choice);

/* One training step on a batch of B samples (all device arrays): features X
 * [B*8], labels y [B] (0 GConn+Euler faster, 1 BFS faster), sample weights w
 * [B].  Loss: mean over samples of w * softmax cross-entropy.  The gradient of
 * the loss (device float [4866], nullable) is written to grad; if adam_m and
 * adam_v (device float [4866] each, zero before step 1) are given and lr > 0,
 * params are updated by Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected
 * with the 1-based step).  loss_host: host float, nullable. */
rst_status rst_mlp_train_step(rst_ctx *ctx, const float *norm, float *params, float *adam_m,
                              float *adam_v, int64_t step, float lr, const float *X,
                              const int32_t *y, const float *w, int64_t B, float *grad,
                              float *loss_host);

/* Load selector weights from a host blob (format above); the context keeps a
 * device copy and uses it when rst_spanning_forest_batch gets method == NULL.
 * RST_E_INVAL on a malformed or non-finite blob. */
rst_status rst_selector_load(rst_ctx *ctx, const void *blob, size_t bytes);

/* Check on the device that parent is a rooted spanning forest of g under the
 * convention of rst_spanning_tree (Sec. I per component: root's component
 * rooted at root, every other one at its minimum id): every entry a vertex id,
 * exactly the designated roots self-parented, every other parent a neighbour,
 * and every vertex reaching its component's root.  *num_failures (host)
 * receives the number of failed checks (0: valid); *first_bad (host, nullable)
 * the smallest failing vertex or -1.  parent: device int32 [n]. */
rst_status rst_verify(rst_ctx *ctx, const rst_csr *g, int32_t root, const int32_t *parent,
                      int64_t *num_failures, int64_t *first_bad);

/* Result of rst_autotune (host struct). */
typedef struct {
  int32_t num_options;    /* entries used in options[] / values[]                 */
  int32_t options[8];     /* rst_option ids of the method's knobs                  */
  int64_t values[8];      /* the chosen value of each (now set on the context)      */
  float ms_best;          /* median time per call with the chosen setting           */
  float ms_default;       /* median time per call with the setting before tuning    */
  int32_t candidates;     /* settings timed besides the starting one                */
  int32_t rejected;       /* settings whose output failed rst_verify (never chosen) */
} rst_tune_result;

/* Autotune the context's tunables for `method` on graph g and root: coordinate
 * descent over the method's knobs (GConn+Euler: sweep block size, hooking
 * heavy degree, ranking words per thread, sparse ruling-set stride; BFS:
 * levels per sync, grid, heavy degree), each candidate timed as the median of
 * `reps` calls (1..101) and rejected unless every call returns the status of
 * the starting setting and its output passes the rst_verify checks against
 * component labels computed once, before the search, with that setting.  The best setting is applied to the context
 * and recorded in its tuning cache under (GPU architecture, method,
 * floor(log2 n), floor(log2 nnz/n)).  Allocates a device buffer of 2n int32
 * for the duration of the call.  result: host, nullable. */
rst_status rst_autotune(rst_ctx *ctx, const rst_csr *g, int32_t root, rst_method method,
                        int32_t reps, rst_tune_result *result);

/* Write the context's tuning cache to a JSON file at host path `path`
 * ({"format": "rst-tune-1", "entries": {key: {"ms": t, "options": {id: value}}}}). */
rst_status rst_tune_save(const rst_ctx *ctx, const char *path);

/* Merge the entries of a JSON tuning cache file into the context's cache; if g
 * is non-NULL and an entry matches (architecture, method, size class of g),
 * apply its setting (*applied = 1, host, nullable).  RST_E_INVAL for a missing
 * or malformed file or an out-of-range value (nothing is applied then). */
rst_status rst_tune_load(rst_ctx *ctx, const char *path, const rst_csr *g, rst_method method,
                         int32_t *applied);

/* Human-readable name of a status code (static string). */
const char *rst_status_string(rst_status s);

#ifdef __cplusplus
}
#endif

#endif /* RST_H */
