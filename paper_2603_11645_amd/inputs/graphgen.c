/*
 * graphgen.c -- seeded synthetic graph construction (host C, OpenMP).
 *
 * This module only builds input graphs: edge lists from counter-based random
 * draws, and a symmetric CSR (sorted neighbour lists, no self-loops, no
 * duplicates) from an edge list.  It computes nothing of the rooted-spanning-
 * tree method itself: no hooking, no pointer jumping, no traversal, no tour.
 * Component restriction and re-connection of the generated graphs are done by
 * the Python layer with scipy's connected-components routine.
 *
 * Random numbers: every draw is rng(seed, stream, index), a pure function of
 * its three arguments built from the splitmix64 finaliser (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), so
 * generation is reproducible and independent of thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t gg_rng(uint64_t seed, uint64_t stream, uint64_t idx) {
  return mix64(mix64(mix64(seed) ^ (stream * 0xD1B54A32D192ED03ull)) + idx);
}

/* uniform double in [0,1) from the top 53 bits */
static inline double gg_unif(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)(gg_rng(seed, stream, idx) >> 11) * (1.0 / 9007199254740992.0);
}

/* Fisher-Yates permutation of 0..n-1 driven by rng(seed, stream, i). */
void gg_permutation(int64_t n, uint64_t seed, uint64_t stream, int32_t *perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)(gg_rng(seed, stream, (uint64_t)i) % (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

/*
 * 4-neighbour grid over the first `limit` cells of a rows x cols row-major
 * layout.  Each right/down edge is deleted independently with probability
 * p_del (draw index 2*cell / 2*cell+1 on `stream`).  If perm is non-NULL the
 * vertex of cell c is perm[c].  Returns the number of edges written (at most
 * 2*limit).
 */
int64_t gg_grid_edges(int64_t rows, int64_t cols, int64_t limit, double p_del,
                      uint64_t seed, uint64_t stream, const int32_t *perm,
                      int32_t *eu, int32_t *ev) {
  int64_t m = 0;
  (void)rows;
  for (int64_t c = 0; c < limit; ++c) {
    int64_t j = c % cols;
    if (j + 1 < cols && c + 1 < limit) {
      if (!(p_del > 0.0 && gg_unif(seed, stream, 2 * (uint64_t)c) < p_del)) {
        eu[m] = perm ? perm[c] : (int32_t)c;
        ev[m] = perm ? perm[c + 1] : (int32_t)(c + 1);
        ++m;
      }
    }
    if (c + cols < limit) {
      if (!(p_del > 0.0 && gg_unif(seed, stream, 2 * (uint64_t)c + 1) < p_del)) {
        eu[m] = perm ? perm[c] : (int32_t)c;
        ev[m] = perm ? perm[c + cols] : (int32_t)(c + cols);
        ++m;
      }
    }
  }
  return m;
}

/*
 * Local diagonals of a rows x cols grid (cells < limit): each candidate
 * (i,j)-(i+1,j+1) and (i,j)-(i+1,j-1) is kept with probability p_diag.
 * Returns the number of edges written (at most 2*limit).
 */
int64_t gg_diag_edges(int64_t rows, int64_t cols, int64_t limit, double p_diag,
                      uint64_t seed, uint64_t stream, int32_t *eu, int32_t *ev) {
  int64_t m = 0;
  (void)rows;
  for (int64_t c = 0; c < limit; ++c) {
    int64_t j = c % cols;
    if (j + 1 < cols && c + cols + 1 < limit &&
        gg_unif(seed, stream, 2 * (uint64_t)c) < p_diag) {
      eu[m] = (int32_t)c; ev[m] = (int32_t)(c + cols + 1); ++m;
    }
    if (j > 0 && c + cols - 1 < limit &&
        gg_unif(seed, stream, 2 * (uint64_t)c + 1) < p_diag) {
      eu[m] = (int32_t)c; ev[m] = (int32_t)(c + cols - 1); ++m;
    }
  }
  return m;
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) endpoint sampling: for each of
 * nsamples edges descend `scale` levels choosing quadrant (0,0),(0,1),(1,0),
 * (1,1) with probabilities a, b, c, 1-a-b-c.  A sample with an endpoint >=
 * n_limit is redrawn (attempt k uses stream base+k).  Writes exactly nsamples
 * edges (self-loops and duplicates are left for the CSR builder to drop).
 */
void gg_rmat_edges(int32_t scale, int64_t nsamples, double a, double b, double c,
                   int64_t n_limit, uint64_t seed, uint64_t stream,
                   int32_t *eu, int32_t *ev) {
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < nsamples; ++s) {
    for (uint64_t attempt = 0;; ++attempt) {
      uint64_t u = 0, v = 0;
      for (int32_t lvl = 0; lvl < scale; ++lvl) {
        double r = gg_unif(seed, stream + 1000003ull * attempt,
                           (uint64_t)s * (uint64_t)scale + (uint64_t)lvl);
        uint64_t ub, vb;
        if (r < a) { ub = 0; vb = 0; }
        else if (r < ab) { ub = 0; vb = 1; }
        else if (r < abc) { ub = 1; vb = 0; }
        else { ub = 1; vb = 1; }
        u = (u << 1) | ub;
        v = (v << 1) | vb;
      }
      if ((int64_t)u < n_limit && (int64_t)v < n_limit) {
        eu[s] = (int32_t)u; ev[s] = (int32_t)v;
        break;
      }
    }
  }
}

/*
 * Long chain: Hamiltonian path perm[0]-perm[1]-...-perm[n-1] plus, at each
 * position i independently with probability p_short, a shortcut to position
 * i+d with d uniform in {2..max_span} (dropped if i+d >= n).
 * eu/ev need room for (n-1) + n edges.  Returns the number written.
 */
int64_t gg_chain_edges(int64_t n, double p_short, int32_t max_span, uint64_t seed,
                       uint64_t stream, const int32_t *perm, int32_t *eu, int32_t *ev) {
  int64_t m = 0;
  for (int64_t i = 0; i + 1 < n; ++i) { eu[m] = perm[i]; ev[m] = perm[i + 1]; ++m; }
  for (int64_t i = 0; i < n; ++i) {
    if (gg_unif(seed, stream, (uint64_t)i) < p_short) {
      int64_t d = 2 + (int64_t)(gg_rng(seed, stream + 1, (uint64_t)i) % (uint64_t)(max_span - 1));
      if (i + d < n) { eu[m] = perm[i]; ev[m] = perm[i + d]; ++m; }
    }
  }
  return m;
}

/*
 * Symmetric CSR from an undirected edge list: both directions stored, self-
 * loops dropped, each neighbour list sorted ascending with duplicates removed.
 * Two stable counting passes (by target, then by source) leave every list
 * sorted without a comparison sort.  off has n+1 entries, cols needs room for
 * 2*m.  Returns nnz, or -1 if scratch memory cannot be allocated.
 */
int64_t gg_build_csr(int64_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                     int64_t *off, int32_t *cols) {
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *bysrc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  if (!cnt || !cur || !bysrc) { free(cnt); free(cur); free(bysrc); return -1; }
  for (int64_t k = 0; k < m; ++k) {
    if (eu[k] == ev[k]) continue;
    cnt[eu[k] + 1]++; cnt[ev[k] + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  /* pass 1: bucket arcs by target; bucket t holds the sources of arcs s->t */
  memcpy(cur, cnt, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t k = 0; k < m; ++k) {
    int32_t u = eu[k], v = ev[k];
    if (u == v) continue;
    bysrc[cur[v]++] = u;   /* arc u->v */
    bysrc[cur[u]++] = v;   /* arc v->u */
  }
  /* pass 2: walk targets ascending and append each to its source's list */
  memcpy(cur, cnt, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t t = 0; t < n; ++t)
    for (int64_t i = cnt[t]; i < cnt[t + 1]; ++i) cols[cur[bysrc[i]]++] = (int32_t)t;
  free(bysrc);
  /* drop duplicates (adjacent after sorting) and compact */
  int64_t pos = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t b = cnt[v], e = cnt[v + 1];
    off[v] = pos;
    for (int64_t i = b; i < e; ++i)
      if (i == b || cols[i] != cols[i - 1]) cols[pos++] = cols[i];
  }
  off[n] = pos;
  free(cnt); free(cur);
  return pos;
}
