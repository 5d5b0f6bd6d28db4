/*
 * oracle.c -- plain, sequential CPU oracle for rooted spanning trees.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test-suite, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code with the HIP library.
 *
 * Paper: "Beyond BFS: A Comparative Study of Rooted Spanning Tree Algorithms
 * on GPUs" (arXiv 2603.11645).  Each function names the passage it follows.
 *
 * Conventions: offsets are int64 [n+1], neighbour ids int32, the CSR is the
 * symmetric adjacency of an undirected graph.  "Designated roots" are the
 * caller's roots; a component holding none of them is rooted at its minimum
 * vertex id.  Every function is single-threaded and allocates its own scratch;
 * a negative return value is an error (-100: out of memory).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ENOMEM (-100)

/* ------------------------------------------------------------------------- */
/* Breadth-first search (Sec. III-A): rounds over frontiers, every vertex of  */
/* distance k is discovered before any of distance k+1.  A FIFO queue over    */
/* neighbours in CSR order gives the hop distance (unique) and the first      */
/* discoverer as parent (one of several valid BFS parents).                   */
/* Returns the largest level reached (eccentricity of root), -1 on bad root.  */
/* ------------------------------------------------------------------------- */
int64_t oracle_bfs(int64_t n, const int64_t *off, const int32_t *cols, int32_t root,
                   int32_t *level, int32_t *parent) {
  if (n < 1 || root < 0 || root >= n) return -1;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return ORC_ENOMEM;
  for (int64_t v = 0; v < n; ++v) { level[v] = -1; parent[v] = -1; }
  int64_t head = 0, tail = 0, ecc = 0;
  level[root] = 0; parent[root] = root; queue[tail++] = root;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t i = off[u]; i < off[u + 1]; ++i) {
      int32_t w = cols[i];
      if (level[w] < 0) {
        level[w] = level[u] + 1;
        parent[w] = u;
        if (level[w] > ecc) ecc = level[w];
        queue[tail++] = w;
      }
    }
  }
  free(queue);
  return ecc;
}

/* union-find with path halving: every visited vertex is re-pointed to its
 * grandparent (the pointer-jumping step P[i] = P[P[i]] of Sec. III-B). */
static int32_t uf_find(int32_t *p, int32_t x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}

/* ------------------------------------------------------------------------- */
/* Connectivity with spanning-edge marking (Sec. III-B "Hooking", with the    */
/* Shiloach-Vishkin bookkeeping of Sec. I): for each undirected edge (u,v),   */
/* taken as the arc u->v with u<v in CSR order, if the roots of u and v       */
/* differ the larger root is linked under the smaller (hooking by vertex id)  */
/* and (u,v) is appended to the forest.  Afterwards label[v] = root of v,     */
/* which is the minimum id of v's component.  fu/fv need room for n-1 edges.  */
/* Returns the number of forest edges t = n - (number of components).         */
/* ------------------------------------------------------------------------- */
int64_t oracle_uf_forest(int64_t n, const int64_t *off, const int32_t *cols,
                         int32_t *label, int32_t *fu, int32_t *fv) {
  if (n < 1) return -1;
  int32_t *p = label;
  for (int64_t v = 0; v < n; ++v) p[v] = (int32_t)v;
  int64_t t = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t i = off[u]; i < off[u + 1]; ++i) {
      int32_t v = cols[i];
      if (v <= u) continue;
      int32_t ru = uf_find(p, (int32_t)u), rv = uf_find(p, v);
      if (ru == rv) continue;
      if (ru < rv) p[rv] = ru; else p[ru] = rv;
      fu[t] = (int32_t)u; fv[t] = v; ++t;
    }
  }
  for (int64_t v = 0; v < n; ++v) label[v] = uf_find(p, (int32_t)v);
  return t;
}

/* min-id component labels of a forest given as an edge list */
static void forest_labels(int64_t n, int64_t t, const int32_t *fu, const int32_t *fv,
                          int32_t *label) {
  for (int64_t v = 0; v < n; ++v) label[v] = (int32_t)v;
  for (int64_t k = 0; k < t; ++k) {
    int32_t a = uf_find(label, fu[k]), b = uf_find(label, fv[k]);
    if (a < b) label[b] = a; else if (b < a) label[a] = b;
  }
  for (int64_t v = 0; v < n; ++v) label[v] = uf_find(label, (int32_t)v);
}

/* Root of every component (Sec. I problem statement, generalised to forests
 * by breaking one cycle per root, Sec. III-D): the designated root if the
 * component holds one, else its minimum id.  is_root[v] = 1 exactly for
 * those vertices.  Returns 0, or -2 for a designated root out of range, -3
 * for two designated roots in one component. */
static int root_flags(int64_t n, const int32_t *label, const int32_t *roots, int32_t nroots,
                      uint8_t *is_root) {
  uint8_t *has = (uint8_t *)calloc((size_t)n, 1);
  if (!has) return ORC_ENOMEM;
  memset(is_root, 0, (size_t)n);
  for (int32_t i = 0; i < nroots; ++i) {
    int32_t r = roots[i];
    if (r < 0 || r >= n) { free(has); return -2; }
    if (has[label[r]]) { free(has); return -3; }
    has[label[r]] = 1;
    is_root[r] = 1;
  }
  for (int64_t v = 0; v < n; ++v)
    if (label[v] == v && !has[v]) is_root[v] = 1;
  free(has);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Rooting a fixed forest at fixed roots (the plain definition behind the RST */
/* problem of Sec. I): P[v] is v's neighbour on the unique tree path from v   */
/* to its component's root, P[root] = root.  Iterative depth-first search     */
/* from each root.  Returns 0 or a negative error (see root_flags).           */
/* ------------------------------------------------------------------------- */
int oracle_dfs_root(int64_t n, int64_t t, const int32_t *fu, const int32_t *fv,
                    const int32_t *roots, int32_t nroots, int32_t *parent) {
  int64_t *adj_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * t + 1));
  int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t *is_root = (uint8_t *)malloc((size_t)n);
  int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int rc = 0;
  if (!adj_off || !adj || !label || !is_root || !stack) { rc = ORC_ENOMEM; goto done; }
  forest_labels(n, t, fu, fv, label);
  rc = root_flags(n, label, roots, nroots, is_root);
  if (rc) goto done;
  for (int64_t k = 0; k < t; ++k) { adj_off[fu[k] + 1]++; adj_off[fv[k] + 1]++; }
  for (int64_t v = 0; v < n; ++v) adj_off[v + 1] += adj_off[v];
  {
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!cur) { rc = ORC_ENOMEM; goto done; }
    memcpy(cur, adj_off, sizeof(int64_t) * (size_t)n);
    for (int64_t k = 0; k < t; ++k) { adj[cur[fu[k]]++] = fv[k]; adj[cur[fv[k]]++] = fu[k]; }
    free(cur);
  }
  for (int64_t v = 0; v < n; ++v) parent[v] = -1;
  for (int64_t r = 0; r < n; ++r) {
    if (!is_root[r]) continue;
    int64_t sp = 0;
    parent[r] = (int32_t)r;
    stack[sp++] = (int32_t)r;
    while (sp) {
      int32_t u = stack[--sp];
      for (int64_t i = adj_off[u]; i < adj_off[u + 1]; ++i) {
        int32_t w = adj[i];
        if (parent[w] < 0) { parent[w] = u; stack[sp++] = w; }
      }
    }
  }
done:
  free(adj_off); free(adj); free(label); free(is_root); free(stack);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Euler-tour rooting, in the order of Sec. III-D.                            */
/*  1. the t forest edges become E = 2t directed arcs: arc k = (fu[k]->fv[k]) */
/*     and arc k+t its reverse, so rev(e) = (e + E/2) mod E;                  */
/*  2. the arcs are sorted lexicographically by (from, to), which makes every */
/*     vertex's out-arcs contiguous; first[v]/last[v] bound that range and    */
/*     next[i] links consecutive arcs with the same source (-1 at the end);   */
/*  3. succ(e) = next(rev e) if that is not -1, else first(from(rev e));      */
/*  4. for every root r with arcs, the successor of the reverse of last[r] is */
/*     set to -1, turning each tree's cycle into a list that starts at        */
/*     first[r];                                                              */
/*  5. every arc is ranked by its position in its list;                       */
/*  6. for each arc e=(u->v) and rev(e)=(v->u): if rank[e] > rank[rev e] then */
/*     e is the return traversal (from child u up to parent v) and            */
/*     P[u] = v, otherwise P[v] = u.  Roots get P[r] = r.                     */
/* Steps 2-6 run in the sorted index space; rev is carried into it through    */
/* the sort permutation.  Optional outputs (indexed by original arc id e):    */
/* succ_out[e] = original id of succ(e) or -1, pos_out[e] = position of e in  */
/* its tour.  Returns 0 or a negative error.                                  */
/* ------------------------------------------------------------------------- */
static const int32_t *g_sort_src, *g_sort_dst;
static int cmp_arc(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  if (g_sort_src[x] != g_sort_src[y]) return g_sort_src[x] < g_sort_src[y] ? -1 : 1;
  if (g_sort_dst[x] != g_sort_dst[y]) return g_sort_dst[x] < g_sort_dst[y] ? -1 : 1;
  return (x > y) - (x < y);
}

int oracle_euler_root(int64_t n, int64_t t, const int32_t *fu, const int32_t *fv,
                      const int32_t *roots, int32_t nroots, int32_t *parent,
                      int32_t *succ_out, int32_t *pos_out) {
  const int64_t E = 2 * t;
  int rc = 0;
  int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
  int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
  int32_t *sorted = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
  int32_t *where = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
  int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
  int32_t *succ = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
  int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
  int32_t *first = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *last = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t *is_root = (uint8_t *)malloc((size_t)n);
  if (!src || !dst || !sorted || !where || !next || !succ || !rank || !first || !last ||
      !label || !is_root) { rc = ORC_ENOMEM; goto done; }
  forest_labels(n, t, fu, fv, label);
  rc = root_flags(n, label, roots, nroots, is_root);
  if (rc) goto done;

  /* 1. arcs and their reverse pairing */
  for (int64_t k = 0; k < t; ++k) {
    src[k] = fu[k]; dst[k] = fv[k];
    src[k + t] = fv[k]; dst[k + t] = fu[k];
  }
  /* 2. lexicographic sort; first/last/next in sorted positions */
  for (int64_t e = 0; e < E; ++e) sorted[e] = (int32_t)e;
  g_sort_src = src; g_sort_dst = dst;
  if (E > 1) qsort(sorted, (size_t)E, sizeof(int32_t), cmp_arc);
  for (int64_t i = 0; i < E; ++i) where[sorted[i]] = (int32_t)i;
  for (int64_t v = 0; v < n; ++v) { first[v] = -1; last[v] = -1; }
  for (int64_t i = 0; i < E; ++i) {
    int32_t s = src[sorted[i]];
    if (first[s] < 0) first[s] = (int32_t)i;
    last[s] = (int32_t)i;
  }
  for (int64_t i = 0; i < E; ++i)
    next[i] = (i < last[src[sorted[i]]]) ? (int32_t)(i + 1) : -1;
  /* 3. successor of every arc (sorted positions) */
  for (int64_t i = 0; i < E; ++i) {
    int32_t e = sorted[i];
    int32_t re = (int32_t)((e + t) % E);           /* rev(e) = (e + E/2) mod E */
    int32_t ri = where[re];
    succ[i] = (next[ri] != -1) ? next[ri] : first[src[re]];
  }
  /* 4. break the cycle of every tree at its root */
  for (int64_t r = 0; r < n; ++r) {
    if (!is_root[r] || last[r] < 0) continue;
    int32_t e_last = sorted[last[r]];
    int32_t re = (int32_t)((e_last + t) % E);
    succ[where[re]] = -1;
  }
  /* 5. rank = position from the head first[r] of each list */
  for (int64_t i = 0; i < E; ++i) rank[i] = -1;
  for (int64_t r = 0; r < n; ++r) {
    if (!is_root[r] || first[r] < 0) continue;
    int32_t i = first[r], p = 0;
    while (i != -1) {
      if (rank[i] != -1 || p > E) { rc = -4; goto done; }  /* not a simple list */
      rank[i] = p++;
      i = succ[i];
    }
  }
  for (int64_t i = 0; i < E; ++i) if (rank[i] < 0) { rc = -4; goto done; }
  /* 6. parents from tour order */
  for (int64_t v = 0; v < n; ++v) parent[v] = is_root[v] ? (int32_t)v : -1;
  for (int64_t e = 0; e < t; ++e) {
    int32_t u = src[e], v = dst[e];
    if (rank[where[e]] > rank[where[e + t]]) parent[u] = v;   /* e returns u -> v */
    else parent[v] = u;                                       /* e descends u -> v */
  }
  if (succ_out)
    for (int64_t e = 0; e < E; ++e) {
      int32_t s = succ[where[e]];
      succ_out[e] = s < 0 ? -1 : sorted[s];
    }
  if (pos_out)
    for (int64_t e = 0; e < E; ++e) pos_out[e] = rank[where[e]];
done:
  free(src); free(dst); free(sorted); free(where); free(next); free(succ); free(rank);
  free(first); free(last); free(label); free(is_root);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Euler successor for an arbitrary per-vertex cyclic order (Sec. III-D; the  */
/* sort only fixes one such order).  Arcs are slots 0..A-1 with twins e, e^1; */
/* a slot with src[e] < 0 is unused and gets succ -1.  head[v] is the first   */
/* out-arc of v (-1 if none), next[e] the following out-arc of src[e] (-1 at  */
/* the end).  succ(e) = next(rev e) if not -1, else head(from(rev e)); then   */
/* for every vertex r with is_root[r] and out-arcs, the last arc of r's list  */
/* is found by walking it and the successor of its reverse is set to -1.      */
/* Returns 0, or -5 if a list is longer than A (malformed input).             */
/* ------------------------------------------------------------------------- */
int oracle_euler_succ(int64_t n, int64_t A, const int32_t *src, const int32_t *dst,
                      const int32_t *head, const int32_t *next, const uint8_t *is_root,
                      int32_t *succ) {
  for (int64_t e = 0; e < A; ++e) {
    if (src[e] < 0) { succ[e] = -1; continue; }
    int32_t re = (int32_t)(e ^ 1);
    succ[e] = (next[re] != -1) ? next[re] : head[src[re]];
  }
  for (int64_t r = 0; r < n; ++r) {
    if (!is_root[r] || head[r] < 0) continue;
    int32_t e = head[r];
    int64_t steps = 0;
    while (next[e] != -1) {
      e = next[e];
      if (++steps > A) return -5;
    }
    succ[e ^ 1] = -1;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* List ranking by a sequential walk (Sec. III-D "parallel list ranking"; the */
/* rank of a node in a list is unique given succ).  dist[e] = number of       */
/* nodes after e in its list (0 at the tail).  Returns the number of lists,   */
/* or -6 if some node lies on a cycle or has two predecessors.                */
/* ------------------------------------------------------------------------- */
int64_t oracle_list_rank(int64_t A, const int32_t *succ, int32_t *dist) {
  uint8_t *has_pred = (uint8_t *)calloc((size_t)A + 1, 1);
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A + 1));
  int64_t lists = 0;
  if (!has_pred || !buf) { free(has_pred); free(buf); return ORC_ENOMEM; }
  for (int64_t e = 0; e < A; ++e) dist[e] = -1;
  for (int64_t e = 0; e < A; ++e) {
    int32_t s = succ[e];
    if (s < -1 || s >= A) { lists = -6; goto done; }
    if (s >= 0) {
      if (has_pred[s]) { lists = -6; goto done; }
      has_pred[s] = 1;
    }
  }
  for (int64_t h = 0; h < A; ++h) {
    if (has_pred[h]) continue;
    int64_t len = 0;
    for (int32_t e = (int32_t)h; e != -1; e = succ[e]) buf[len++] = e;
    for (int64_t i = 0; i < len; ++i) dist[buf[i]] = (int32_t)(len - 1 - i);
    ++lists;
  }
  for (int64_t e = 0; e < A; ++e) if (dist[e] < 0) { lists = -6; goto done; }
done:
  free(has_pred); free(buf);
  return lists;
}

/* ------------------------------------------------------------------------- */
/* Verifier of the RST definition of Sec. I, per component:                   */
/*  1. P[r] = r for every root (designated, or min id of a component with no  */
/*     designated root);                                                      */
/*  2. 0 <= P[v] < n;                                                         */
/*  3. {v, P[v]} is an edge of G for every non-root v;                        */
/*  4. following P from any v ends at a root without revisiting a vertex;     */
/*  5. that root is the root of v's component.                                */
/* Together: P is a spanning forest of G made of graph edges, one tree per    */
/* component, each rooted where required.  Returns 0 if valid, else the code  */
/* of the first failed check (1..5; 6 for bad designated roots) and the       */
/* offending vertex in *bad.                                                  */
/* ------------------------------------------------------------------------- */
int oracle_verify_rst(int64_t n, const int64_t *off, const int32_t *cols,
                      const int32_t *parent, const int32_t *roots, int32_t nroots,
                      int64_t *bad) {
  int rc = 0;
  int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fu = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t *is_root = (uint8_t *)malloc((size_t)n);
  int32_t *state = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);   /* -2 new, -1 on path, >=0 root */
  int32_t *pathbuf = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  *bad = -1;
  if (!label || !fu || !fv || !is_root || !state || !pathbuf) { rc = ORC_ENOMEM; goto done; }
  if (oracle_uf_forest(n, off, cols, label, fu, fv) < 0) { rc = 6; goto done; }
  if (root_flags(n, label, roots, nroots, is_root)) { rc = 6; goto done; }
  for (int64_t v = 0; v < n; ++v) {
    if (is_root[v] && parent[v] != v) { rc = 1; *bad = v; goto done; }
    if (parent[v] < 0 || parent[v] >= n) { rc = 2; *bad = v; goto done; }
  }
  for (int64_t v = 0; v < n; ++v) {
    if (is_root[v]) continue;
    int32_t p = parent[v];
    int found = 0;
    for (int64_t i = off[v]; i < off[v + 1]; ++i) if (cols[i] == p) { found = 1; break; }
    if (!found) { rc = 3; *bad = v; goto done; }
  }
  for (int64_t v = 0; v < n; ++v) state[v] = -2;
  for (int64_t v = 0; v < n; ++v) {
    if (state[v] != -2) continue;
    int64_t len = 0;
    int32_t x = (int32_t)v, reached;
    for (;;) {
      if (state[x] >= 0) { reached = state[x]; break; }
      if (state[x] == -1) { rc = 4; *bad = x; goto done; }   /* cycle */
      state[x] = -1;
      pathbuf[len++] = x;
      if (parent[x] == x) { reached = x; break; }
      x = parent[x];
    }
    for (int64_t i = 0; i < len; ++i) state[pathbuf[i]] = reached;
  }
  for (int64_t v = 0; v < n; ++v) {
    int32_t r = state[v];
    if (!is_root[r] || label[r] != label[v]) { rc = 5; *bad = v; goto done; }
  }
done:
  free(label); free(fu); free(fv); free(is_root); free(state); free(pathbuf);
  return rc;
}

/* Component count and min-id labels only (convenience for tests). */
int64_t oracle_components(int64_t n, const int64_t *off, const int32_t *cols, int32_t *label) {
  int32_t *fu = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!fu || !fv) { free(fu); free(fv); return ORC_ENOMEM; }
  int64_t t = oracle_uf_forest(n, off, cols, label, fu, fv);
  free(fu); free(fv);
  return t < 0 ? t : n - t;
}

/* ------------------------------------------------------------------------- */
/* Depth of every vertex in a rooted forest (the tree-depth property compared */
/* across methods in Sec. IV-B, Fig. 2): depth[v] = number of parent steps    */
/* from v to the root of its tree (P[root] = root, depth 0).  Plain walk up   */
/* the parent pointers with memoisation.  Returns the largest depth, -7 for a */
/* parent out of range, -8 for a cycle.                                       */
/* ------------------------------------------------------------------------- */
int64_t oracle_tree_depth(int64_t n, const int32_t *parent, int32_t *depth) {
  int32_t *path = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!path) return ORC_ENOMEM;
  int64_t maxd = 0, rc = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (parent[v] < 0 || parent[v] >= n) { rc = -7; goto done; }
    depth[v] = -1;
  }
  for (int64_t v = 0; v < n; ++v) {
    if (depth[v] >= 0) continue;
    int64_t len = 0;
    int32_t x = (int32_t)v;
    /* climb until a vertex of known depth or a root; -2 marks "on this walk" */
    while (depth[x] == -1 && parent[x] != x) {
      depth[x] = -2;
      path[len++] = x;
      x = parent[x];
    }
    if (depth[x] == -2) { rc = -8; goto done; }
    if (depth[x] == -1) depth[x] = 0;          /* x is a root */
    int32_t d = depth[x];
    for (int64_t i = len - 1; i >= 0; --i) depth[path[i]] = ++d;
    if (d > maxd) maxd = d;
  }
  rc = maxd;
done:
  free(path);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Path-Reversal RST (Sec. III-C, after Cong and Bader), sequential, in the   */
/* order of the paper.  A rooted spanning forest P (every vertex its own root */
/* at the start) is kept at all times.  Each iteration:                       */
/*  1. pointer jumping with history: anc[0] = P, anc[k+1][v] =                */
/*     anc[k][anc[k][v]] for K = ceil(log2 n) + 1 levels (the "special        */
/*     ancestors" at distances 2^k); rep[v] = anc[K-1][v], the root of v;     */
/*  2. hooking, alternating max and min: on even iterations the component of  */
/*     the larger representative is the target of every edge joining two      */
/*     components, on odd ones the smaller; the other root r gets one hooking */
/*     edge (x in r's tree, y in the target's tree); here the first such arc  */
/*     in CSR order wins (on the GPU any may);                                */
/*  3. path marking: x is on the path, and in round k = 0..K-1 every marked   */
/*     vertex marks its 2^k-th ancestor (all marked vertices are ancestors    */
/*     of x, so marking within a round is harmless);                          */
/*  4. reversal: for every marked non-root v, P'[P[v]] = v; then P'[x] = y    */
/*     grafts r's tree, re-rooted at x, onto y.                               */
/* The loop ends when no edge joins two components.  Finally every tree is    */
/* re-rooted at its designated root d, or at its minimum id if it holds none, */
/* by the same marking and reversal (P'[d] = d).                              */
/* Returns the number of hooking iterations, or a negative error (see         */
/* root_flags; -9 if the iteration cap 4 n + 64 is exceeded).  max_iters >= 0 */
/* stops after that many iterations and returns the forest as it stands, not  */
/* re-rooted (for checking single steps).                                     */
/* ------------------------------------------------------------------------- */
static int ceil_log2_levels(int64_t n) {
  int k = 1;
  while (((int64_t)1 << (k - 1)) < n) ++k;
  return k;
}

/* anc[k] for k < K (anc + k*n), from P */
static void special_ancestors(int64_t n, int K, const int32_t *P, int32_t *anc) {
  memcpy(anc, P, sizeof(int32_t) * (size_t)n);
  for (int k = 1; k < K; ++k) {
    const int32_t *a = anc + (size_t)(k - 1) * (size_t)n;
    int32_t *b = anc + (size_t)k * (size_t)n;
    for (int64_t v = 0; v < n; ++v) b[v] = a[a[v]];
  }
}

/* mark the tree path from every start vertex (on[v] = 1 already) to its root */
static void mark_paths(int64_t n, int K, const int32_t *anc, uint8_t *on) {
  for (int k = 0; k < K; ++k) {
    const int32_t *a = anc + (size_t)k * (size_t)n;
    for (int64_t v = 0; v < n; ++v)
      if (on[v]) on[a[v]] = 1;
  }
}

int64_t oracle_pr_rst(int64_t n, const int64_t *off, const int32_t *cols, const int32_t *roots,
                      int32_t nroots, int64_t max_iters, int32_t *parent) {
  const int K = ceil_log2_levels(n);
  int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)K);
  int32_t *np = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *wx = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *wy = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t *on = (uint8_t *)malloc((size_t)n);
  int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fu = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t *is_root = (uint8_t *)malloc((size_t)n);
  int64_t iters = 0;
  if (!anc || !np || !wx || !wy || !on || !label || !fu || !fv || !is_root) { iters = ORC_ENOMEM; goto done; }
  /* designated roots are checked first (two in one component is an error) */
  if (oracle_uf_forest(n, off, cols, label, fu, fv) < 0) { iters = -1; goto done; }
  { int rc = root_flags(n, label, roots, nroots, is_root); if (rc) { iters = rc; goto done; } }
  for (int64_t v = 0; v < n; ++v) parent[v] = (int32_t)v;
  for (;;) {
    if (max_iters >= 0 && iters >= max_iters) goto done;          /* stop early: no re-rooting */
    if (iters > 4 * n + 64) { iters = -9; goto done; }
    special_ancestors(n, K, parent, anc);                          /* step 1 */
    const int32_t *rep = anc + (size_t)(K - 1) * (size_t)n;
    const int max_round = (iters % 2) == 0;
    int64_t hooks = 0;
    for (int64_t v = 0; v < n; ++v) wx[v] = -1;
    for (int64_t u = 0; u < n; ++u) {                              /* step 2 */
      for (int64_t i = off[u]; i < off[u + 1]; ++i) {
        const int32_t w = cols[i];
        const int32_t ru = rep[u], rw = rep[w];
        if (ru == rw) continue;
        const int32_t target = max_round ? (ru > rw ? ru : rw) : (ru < rw ? ru : rw);
        const int32_t r = target == ru ? rw : ru;                  /* the root that is grafted */
        if (wx[r] >= 0) continue;
        wx[r] = target == ru ? w : (int32_t)u;                     /* endpoint in r's tree */
        wy[r] = target == ru ? (int32_t)u : w;                     /* endpoint in the target's */
        ++hooks;
      }
    }
    if (hooks == 0) break;
    memset(on, 0, (size_t)n);                                      /* step 3 */
    for (int64_t r = 0; r < n; ++r) if (wx[r] >= 0) on[wx[r]] = 1;
    mark_paths(n, K, anc, on);
    memcpy(np, parent, sizeof(int32_t) * (size_t)n);               /* step 4 */
    for (int64_t v = 0; v < n; ++v)
      if (on[v] && parent[v] != v) np[parent[v]] = (int32_t)v;
    for (int64_t r = 0; r < n; ++r) if (wx[r] >= 0) np[wx[r]] = wy[r];
    memcpy(parent, np, sizeof(int32_t) * (size_t)n);
    ++iters;
  }
  /* re-root every tree at its designated root, or at its minimum id */
  special_ancestors(n, K, parent, anc);
  memcpy(on, is_root, (size_t)n);
  mark_paths(n, K, anc, on);
  memcpy(np, parent, sizeof(int32_t) * (size_t)n);
  for (int64_t v = 0; v < n; ++v)
    if (on[v] && parent[v] != v) np[parent[v]] = (int32_t)v;
  for (int64_t v = 0; v < n; ++v) if (is_root[v]) np[v] = (int32_t)v;
  memcpy(parent, np, sizeof(int32_t) * (size_t)n);
done:
  free(anc); free(np); free(wx); free(wy); free(on); free(label); free(fu); free(fv); free(is_root);
  return iters;
}

/* ------------------------------------------------------------------------- */
/* Biconnected components: the downstream use of a rooted spanning tree that */
/* Sec. I and the opening of Sec. IV name (Tarjan and Vishkin's parallel     */
/* method takes an RST as input).  The oracle is the sequential depth-first  */
/* method of Hopcroft and Tarjan: edges are stacked as the search meets them; */
/* when the search returns from child w to its parent p with low[w] >=       */
/* pre[p], the edges stacked since the tree edge p->w, that edge included,   */
/* form one component, and p is an articulation point unless it roots the    */
/* search (a root is one when it has two or more search children).           */
/* Every undirected edge copy is stacked once (from the side where the other  */
/* end was seen first); the reverse arcs take the label of a stacked arc     */
/* between the same two vertices (parallel copies lie on a common 2-cycle, so */
/* they share a component).  Self-loops get -1.                               */
/* arc_label[nnz] in [0, components), art[n] in {0, 1}.  Returns the number   */
/* of components.                                                             */
/* ------------------------------------------------------------------------- */
static int cmp_u64(const void *a, const void *b) {
  const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

int64_t oracle_bcc(int64_t n, const int64_t *off, const int32_t *cols, int32_t *arc_label,
                   uint8_t *art) {
  const int64_t nnz = off[n];
  int64_t *pre = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *low = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *it = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *pa = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));     /* arc entering v */
  int32_t *par = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  uint8_t *skipped = calloc((size_t)(n > 0 ? n : 1), 1);
  int32_t *vs = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));     /* vertex stack */
  int64_t *es = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1)); /* edge stack */
  int64_t comps = 0;
  if (!pre || !low || !it || !pa || !par || !skipped || !vs || !es) { comps = ORC_ENOMEM; goto done; }
  for (int64_t v = 0; v < n; ++v) { pre[v] = -1; art[v] = 0; }
  for (int64_t a = 0; a < nnz; ++a) arc_label[a] = -1;
  int64_t clock = 0;
  for (int64_t s = 0; s < n; ++s) {
    if (pre[s] >= 0) continue;
    int64_t top = 0, etop = 0, root_children = 0;
    pre[s] = low[s] = clock++;
    it[s] = off[s];
    par[s] = -1;
    pa[s] = -1;
    vs[top++] = (int32_t)s;
    while (top > 0) {
      const int32_t u = vs[top - 1];
      if (it[u] < off[u + 1]) {
        const int64_t a = it[u]++;
        const int32_t w = cols[a];
        if (w == u) continue;                                    /* self-loop */
        if (pre[w] < 0) {                                        /* tree edge */
          es[etop++] = a;
          pre[w] = low[w] = clock++;
          it[w] = off[w];
          par[w] = u;
          pa[w] = a;
          vs[top++] = w;
          if (u == s) ++root_children;
        } else if (pre[w] < pre[u]) {
          if (w == par[u] && !skipped[u]) { skipped[u] = 1; continue; }  /* the tree edge back */
          es[etop++] = a;                                        /* back edge */
          if (pre[w] < low[u]) low[u] = pre[w];
        }
        /* pre[w] > pre[u]: a descendant's edge, stacked from its side */
      } else {
        --top;
        if (u == s) break;
        const int32_t p = par[u];
        if (low[u] < low[p]) low[p] = low[u];
        if (low[u] >= pre[p]) {
          int64_t e;
          do {
            e = es[--etop];
            arc_label[e] = (int32_t)comps;
          } while (e != pa[u]);
          ++comps;
          if (p != s) art[p] = 1;
        }
      }
    }
    if (root_children >= 2) art[s] = 1;
  }
  /* the arcs not stacked take the label of a stacked arc between the same
     ends: (pair key, label) entries sorted by key, then a binary search */
  {
    int64_t k = 0;
    for (int64_t a = 0; a < nnz; ++a) k += arc_label[a] >= 0;
    uint64_t *pk = malloc(sizeof(uint64_t) * 2 * (size_t)(k > 0 ? k : 1));
    if (!pk) { comps = ORC_ENOMEM; goto done; }
    k = 0;
    for (int64_t u = 0; u < n; ++u)
      for (int64_t a = off[u]; a < off[u + 1]; ++a) {
        if (arc_label[a] < 0) continue;
        const uint64_t x = (uint64_t)u, y = (uint64_t)(uint32_t)cols[a];
        pk[2 * k] = (x < y ? x : y) * (uint64_t)n + (x < y ? y : x);
        pk[2 * k + 1] = (uint64_t)(uint32_t)arc_label[a];
        ++k;
      }
    qsort(pk, (size_t)k, 2 * sizeof(uint64_t), cmp_u64);   /* by the pair key */
    for (int64_t u = 0; u < n; ++u)
      for (int64_t a = off[u]; a < off[u + 1]; ++a) {
        const int32_t w = cols[a];
        if (arc_label[a] >= 0 || w == (int32_t)u) continue;
        const uint64_t x = (uint64_t)u, y = (uint64_t)(uint32_t)w;
        const uint64_t key = (x < y ? x : y) * (uint64_t)n + (x < y ? y : x);
        int64_t lo = 0, hi = k;                                  /* first entry >= key */
        while (lo < hi) {
          const int64_t mid = (lo + hi) / 2;
          if (pk[2 * mid] < key) lo = mid + 1; else hi = mid;
        }
        if (lo < k && pk[2 * lo] == key) arc_label[a] = (int32_t)pk[2 * lo + 1];
      }
    free(pk);
  }
done:
  free(pre); free(low); free(it); free(pa); free(par); free(skipped); free(vs); free(es);
  return comps;
}
