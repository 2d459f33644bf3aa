/*
 * CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded, slow reference for the RCM-relabelled
 * direction-optimizing BFS of "Fast and Efficient Parallel Breadth-First
 * Search with Power-law Graph Transformation" (Jiang et al., PPoPP'21
 * poster).  Only the tests, the package's smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code with the GPU library.
 *
 * Graphs are canonical undirected CSR (section 3.1, Eq. 2): off[n+1] int64,
 * cols[nnz] int32, every edge stored in both directions, rows ascending,
 * no self-loops, no duplicates.  deg(v) = off[v+1] - off[v].
 *
 * Functions and the passages they follow:
 *   orc_bandwidth         Eq. 1 (matrix bandwidth), in a given labelling.
 *   orc_canonical_csr     section 3.1 / Eq. 2: CSR of the undirected edge set.
 *   orc_rcm               RCM (section 3.2, Algorithm 3) from its definition:
 *                         the Cuthill-McKee order is a breadth-first search
 *                         per component from its vertex of least
 *                         (degree, id), children queued in (degree, id)
 *                         order; that order reversed, isolated vertices
 *                         appended in increasing id.
 *   orc_rcm_partial       section 4.6 (partial RCM): Algorithm 3 cut off after
 *                         a given number of vertices (reading stated at the
 *                         function).
 *   orc_bfs               Algorithms 1-2 output: hop distance from the source
 *                         and the predecessor map (pi(s) = s, -1 when
 *                         unreachable) with the maximum-label parent rule.
 *   orc_level_counters    per-level frontier / unvisited sizes that drive the
 *                         direction switch of Algorithm 2 and the work the
 *                         bottom-up step of Algorithm 2 / 5 does.
 *   orc_heuristic_schedule the alpha/beta direction rule (section 2.1 and
 *                         "Parameter Tuning"), integer form.
 *   orc_certify_bfs       O(nnz) certificate that (depth, parent) is the
 *                         unique BFS result under the maximum-label rule.
 *   orc_certify_rcm       O(nnz) certificate that a permutation is exactly
 *                         the one Algorithm 3 produces.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Eq. 1: BW(A) = max { i - j : A_ij != 0, i > j }, with vertex v carrying
 * label ell[v] (identity if ell is NULL). */
int64_t orc_bandwidth(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* ell) {
  int64_t bw = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t i = ell ? ell[v] : v;
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
      int64_t j = ell ? ell[cols[e]] : cols[e];
      if (i > j && i - j > bw) bw = i - j;
    }
  }
  return bw;
}

/* ------------------------------------------------------------------------ */
/* Canonical CSR of the undirected edge set {{u, v} : (u, v) a tuple, u != v}.
 * Writes off[n+1] and cols (capacity 2m); returns nnz. */
static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

int64_t orc_canonical_csr(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                          int64_t* off, int32_t* cols) {
  uint64_t* pairs = (uint64_t*)malloc(sizeof(uint64_t) * (2 * m + 1));
  int64_t np = 0;
  for (int64_t i = 0; i < m; ++i) {
    uint64_t u = (uint32_t)src[i], v = (uint32_t)dst[i];
    if (u == v) continue;
    pairs[np++] = (u << 32) | v;
    pairs[np++] = (v << 32) | u;
  }
  qsort(pairs, (size_t)np, sizeof(uint64_t), cmp_u64);
  int64_t nnz = 0;
  for (int64_t v = 0; v <= n; ++v) off[v] = 0;
  for (int64_t i = 0; i < np; ++i) {
    if (i > 0 && pairs[i] == pairs[i - 1]) continue;
    cols[nnz++] = (int32_t)(pairs[i] & 0xFFFFFFFFu);
    off[(pairs[i] >> 32) + 1] += 1;
  }
  for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
  free(pairs);
  return nnz;
}

/* ------------------------------------------------------------------------ */
/* Cuthill-McKee order (section 3.2), written from its definition: the
 * vertices of V+ are visited by one breadth-first search per connected
 * component.  A search starts at the not yet placed vertex of least
 * (degree, id) -- "increasing degree" with ties to the smaller id -- and
 * every vertex taken out of the FIFO queue puts its not yet placed
 * neighbours into the queue in increasing (degree, id).  The order in which
 * vertices leave the queue is the Cuthill-McKee sequence.  Reversing it
 * gives RCM (Algorithm 3).  The order "increasing degree" is read as
 * increasing (degree, vertex id) throughout. */
static _Thread_local const int64_t* g_sort_off; /* degree lookup for the comparator */

static int cmp_deg_id(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  int64_t dx = g_sort_off[x + 1] - g_sort_off[x];
  int64_t dy = g_sort_off[y + 1] - g_sort_off[y];
  if (dx != dy) return dx < dy ? -1 : 1;
  return (x > y) - (x < y);
}

/* seq[0..returned) = the first min(limit, n+) vertices of the Cuthill-McKee
 * sequence; *nplus_out = n+ = |V+|. */
static int64_t cm_sequence(int64_t n, const int64_t* off, const int32_t* cols, int64_t limit,
                           int32_t* seq, int64_t* nplus_out) {
  g_sort_off = off;
  /* candidate starts: the non-isolated vertices in increasing (degree, id) */
  int32_t* starts = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  int64_t nplus = 0;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] > off[v]) starts[nplus++] = (int32_t)v;
  qsort(starts, (size_t)nplus, sizeof(int32_t), cmp_deg_id);
  if (limit > nplus) limit = nplus;

  char* queued = (char*)calloc((size_t)n + 1, 1);    /* ever put in the queue */
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  int32_t* kids = (int32_t*)malloc(sizeof(int32_t) * (n + 1)); /* one vertex's new children */
  int64_t out = 0;
  for (int64_t s = 0; s < nplus && out < limit; ++s) {
    const int32_t start = starts[s];
    if (queued[start]) continue; /* already in an earlier component */
    int64_t head = 0, tail = 0;
    queue[tail++] = start;
    queued[start] = 1;
    while (head < tail && out < limit) {
      const int32_t u = queue[head++];
      seq[out++] = u;
      int64_t nk = 0;
      for (int64_t e = off[u]; e < off[u + 1]; ++e)
        if (!queued[cols[e]]) kids[nk++] = cols[e];
      qsort(kids, (size_t)nk, sizeof(int32_t), cmp_deg_id);
      for (int64_t j = 0; j < nk; ++j) {
        queued[kids[j]] = 1;
        queue[tail++] = kids[j];
      }
    }
  }
  free(kids);
  free(queue);
  free(queued);
  free(starts);
  *nplus_out = nplus;
  return out;
}

/* iperm[k] = original vertex that receives label k; perm[v] = label of v.
 * RCM gives sequence position j of the Cuthill-McKee order the label
 * n+ - 1 - j (the reversal), and the isolated vertices the labels n+ .. n-1
 * in increasing id.  Returns n+ = |V+|, the number of non-isolated
 * vertices. */
int64_t orc_rcm(int64_t n, const int64_t* off, const int32_t* cols, int32_t* iperm,
                int32_t* perm) {
  int64_t nplus = 0;
  int32_t* seq = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  cm_sequence(n, off, cols, n, seq, &nplus);
  for (int64_t j = 0; j < nplus; ++j) iperm[nplus - 1 - j] = seq[j];
  int64_t k = nplus;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] == off[v]) iperm[k++] = (int32_t)v;
  for (int64_t i = 0; i < n; ++i) perm[iperm[i]] = (int32_t)i;
  free(seq);
  return nplus;
}

/* Partial RCM (section 4.6): only part of the vertices is reordered.
 * Reading: the first `keep` vertices of the Cuthill-McKee sequence take
 * labels [0, keep) in reverse sequence order; the other non-isolated
 * vertices follow in increasing id (their order is left alone); the
 * isolated vertices come last in increasing id.  keep >= n+ is Algorithm 3
 * itself; keep = 0 only moves the isolated vertices to the end.  A ratio p
 * of the section maps to keep = ceil(p * n+).  Returns n+. */
int64_t orc_rcm_partial(int64_t n, const int64_t* off, const int32_t* cols, int64_t keep,
                        int32_t* iperm, int32_t* perm) {
  int64_t nplus = 0;
  int32_t* seq = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  const int64_t placed = cm_sequence(n, off, cols, keep < 0 ? 0 : keep, seq, &nplus);
  char* in_seq = (char*)calloc((size_t)n + 1, 1);
  for (int64_t j = 0; j < placed; ++j) {
    iperm[placed - 1 - j] = seq[j];
    in_seq[seq[j]] = 1;
  }
  int64_t k = placed;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] > off[v] && !in_seq[v]) iperm[k++] = (int32_t)v;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] == off[v]) iperm[k++] = (int32_t)v;
  for (int64_t i = 0; i < n; ++i) perm[iperm[i]] = (int32_t)i;
  free(in_seq);
  free(seq);
  return nplus;
}

/* ------------------------------------------------------------------------ */
/* BFS result.  depth[v] = hop distance from root (-1 if unreachable);
 * parent[root] = root; parent[v] = the neighbour u with depth[u] =
 * depth[v] - 1 of largest label ell[u] (identity labels if ell is NULL);
 * parent[v] = -1 if unreachable.  Returns the number of levels (max depth+1).
 * The predecessor map of sections 2.1 and Algorithms 1-2 may name any
 * neighbour one level up; fixing the largest label makes it unique, and is
 * the neighbour that the degree-ordered bottom-up scan of Algorithm 6 meets
 * first once labels rise with degree (after RCM). */
int32_t orc_bfs(int64_t n, const int64_t* off, const int32_t* cols, int32_t root,
                const int32_t* ell, int32_t* depth, int32_t* parent) {
  for (int64_t v = 0; v < n; ++v) {
    depth[v] = -1;
    parent[v] = -1;
  }
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  int64_t head = 0, tail = 0;
  depth[root] = 0;
  queue[tail++] = root;
  int32_t maxd = 0;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t w = cols[e];
      if (depth[w] < 0) {
        depth[w] = depth[u] + 1;
        if (depth[w] > maxd) maxd = depth[w];
        queue[tail++] = w;
      }
    }
  }
  free(queue);
  for (int64_t v = 0; v < n; ++v) {
    if (depth[v] <= 0) continue;
    int32_t best = -1;
    int64_t best_label = INT64_MIN;
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
      int32_t u = cols[e];
      if (depth[u] == depth[v] - 1) {
        int64_t lab = ell ? ell[u] : u;
        if (lab > best_label) {
          best_label = lab;
          best = u;
        }
      }
    }
    parent[v] = best;
  }
  parent[root] = root;
  return maxd + 1;
}

/* ------------------------------------------------------------------------ */
/* Per-level counters for levels d = 0 .. nlev-1 (arrays of length nlev):
 *   nf[d]  = |F_d|, F_d = {v : depth[v] = d}
 *   mf[d]  = sum of deg over F_d
 *   nu[d]  = |U_d|, U_d = {v in the swept set : depth[v] > d or unreached}
 *   mu[d]  = sum of deg over U_d
 *   ebu[d] = edges a bottom-up pass over U_d examines when every row is
 *            scanned in decreasing label order and stops at the first
 *            neighbour in F_d: 1 + (number of neighbours of larger label
 *            than that neighbour), or deg(v) when there is none.
 *   ebc[d] = the part of ebu[d] spent on vertices of the root's component
 *            (those reached later, depth > d): a bottom-up pass needs to
 *            sweep only that component, since a vertex of another one has
 *            no neighbour in F_d and is never reached.
 * The swept set is the first n_sweep vertices in label order (the
 * non-isolated prefix after RCM, or every vertex without it). */
void orc_level_counters(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* ell,
                        int64_t n_sweep, const int32_t* depth, int32_t nlev, int64_t* nf,
                        int64_t* mf, int64_t* nu, int64_t* mu, int64_t* ebu, int64_t* ebc) {
  for (int32_t d = 0; d < nlev; ++d) {
    nf[d] = mf[d] = nu[d] = mu[d] = ebu[d] = ebc[d] = 0;
  }
  for (int64_t v = 0; v < n; ++v) {
    int64_t lab = ell ? ell[v] : v;
    int64_t dv = depth[v];
    int64_t deg = off[v + 1] - off[v];
    if (dv >= 0 && dv < nlev) {
      nf[dv] += 1;
      mf[dv] += deg;
    }
    if (lab >= n_sweep) continue;
    for (int32_t d = 0; d < nlev; ++d) {
      if (dv >= 0 && dv <= d) continue; /* reached by level d */
      nu[d] += 1;
      mu[d] += deg;
      /* bottom-up work on v at level d */
      int64_t first = INT64_MIN;
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        int32_t w = cols[e];
        int64_t lw = ell ? ell[w] : w;
        if (depth[w] == d && lw > first) first = lw;
      }
      int64_t work = deg;
      if (first != INT64_MIN) {
        int64_t larger = 0;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
          int32_t w = cols[e];
          int64_t lw = ell ? ell[w] : w;
          if (lw > first) larger++;
        }
        work = 1 + larger;
      }
      ebu[d] += work;
      if (dv >= 0) ebc[d] += work;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Direction rule (0 = top-down, 1 = bottom-up) for levels 0 .. nlev-1, where
 * level d expands F_d.  Level 0 is top-down.  For d >= 1, with the counters
 * of F_d and U_d:
 *   top-down  -> bottom-up  if mf[d] * alpha > mu[d]
 *   bottom-up -> top-down   if nf[d] * beta < n_sweep and nf[d] < nf[d-1]
 *   otherwise the direction is kept. */
void orc_heuristic_schedule(int32_t nlev, const int64_t* nf, const int64_t* mf,
                            const int64_t* mu, int64_t n_sweep, int64_t alpha, int64_t beta,
                            int8_t* dir) {
  if (nlev <= 0) return;
  dir[0] = 0;
  for (int32_t d = 1; d < nlev; ++d) {
    int8_t prev = dir[d - 1];
    int8_t next = prev;
    if (prev == 0) {
      if (mf[d] * alpha > mu[d]) next = 1;
    } else {
      if (nf[d] * beta < n_sweep && nf[d] < nf[d - 1]) next = 0;
    }
    dir[d] = next;
  }
}

/* ------------------------------------------------------------------------ */
/* BFS certificate.  Returns 0 when (depth, parent) is the BFS result from
 * root under the maximum-label parent rule, else a negative code naming the
 * first failed rule:
 *   -1 root entries wrong            -2 an edge joins reached and unreached
 *   -3 an edge spans > 1 level        -4 unreached vertex with a parent
 *   -5 parent not a neighbour one level up
 *   -6 a neighbour one level up has a larger label than the parent
 *   -7 depth/parent out of range.
 * Rules: the parent chain gives depth >= distance; the edge rule gives
 * depth <= distance; so depth is the distance and the reached set is the
 * component, and the parent is the unique maximum. */
int32_t orc_certify_bfs(int64_t n, const int64_t* off, const int32_t* cols, int32_t root,
                        const int32_t* ell, const int32_t* depth, const int32_t* parent) {
  if (root < 0 || root >= n) return -7;
  if (depth[root] != 0 || parent[root] != root) return -1;
  for (int64_t v = 0; v < n; ++v) {
    int32_t dv = depth[v];
    if (dv < -1 || parent[v] < -1 || parent[v] >= n) return -7;
    if (dv == -1 && parent[v] != -1) return -4;
    if (dv == 0 && v != root) return -1;
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
      int32_t dw = depth[cols[e]];
      if ((dv < 0) != (dw < 0)) return -2;
      if (dv >= 0 && (dv - dw > 1 || dw - dv > 1)) return -3;
    }
    if (dv > 0) {
      int32_t p = parent[v];
      if (p < 0 || depth[p] != dv - 1) return -5;
      int found = 0;
      int64_t lp = ell ? ell[p] : p;
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        int32_t w = cols[e];
        if (w == p) found = 1;
        if (depth[w] == dv - 1) {
          int64_t lw = ell ? ell[w] : w;
          if (lw > lp) return -6;
        }
      }
      if (!found) return -5;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* RCM certificate.  Returns 0 iff perm is exactly Algorithm 3's permutation
 * (under the (degree, id) reading of its orderings), else a negative code.
 *
 * Let n+ = |V+|, cm(v) = n+ - 1 - perm[v] the label before reversal and
 * order[k] the vertex with cm = k.  Algorithm 3 labels vertex k as follows:
 * if some already-labelled vertex still has an unlabelled neighbour, take the
 * smallest label j with one, and give k to the unlabelled neighbour of
 * order[j] with the least (degree, id); otherwise k starts a new component
 * and goes to the unlabelled vertex of least (degree, id).  Equivalently,
 * with p(v) = min cm over N(v) and M(k) = max cm over the neighbours of
 * labels < k:
 *   (a) M(k) < k  (nothing pending): order[k] has the least (degree, id)
 *       among labels >= k;
 *   (b) M(k) >= k: p(order[k]) < k, and over these "appended" vertices the
 *       key (p(v), degree, id) strictly increases with the label.
 *   (c) isolated vertices hold labels n+ .. n-1 in increasing id.
 * Codes: -1 not a bijection, -2 isolated placement, -3 start not minimal,
 *        -4 appended vertex without an earlier neighbour, -5 appended order. */
int32_t orc_certify_rcm(int64_t n, const int64_t* off, const int32_t* cols,
                        const int32_t* perm) {
  int32_t rc = 0;
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  int32_t* cm = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  uint64_t* sufmin = (uint64_t*)malloc(sizeof(uint64_t) * (n + 2));
  for (int64_t k = 0; k < n; ++k) order[k] = -1;
  for (int64_t v = 0; v < n; ++v) {
    if (perm[v] < 0 || perm[v] >= n || order[perm[v]] != -1) { rc = -1; goto done; }
    order[perm[v]] = (int32_t)v;
  }
  int64_t nplus = 0;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] > off[v]) nplus++;
  {
    int64_t k = nplus;
    for (int64_t v = 0; v < n; ++v) {
      if (off[v + 1] == off[v]) {
        if (perm[v] != k) { rc = -2; goto done; }
        k++;
      }
    }
  }
  /* cm labels: order_cm[k] = order[n+ - 1 - k] */
  for (int64_t k = 0; k < nplus; ++k) {
    int32_t v = order[nplus - 1 - k];
    cm[v] = (int32_t)k;
  }
  /* key(v) = deg << 32 | id ; suffix minimum over cm labels >= k */
  sufmin[nplus] = UINT64_MAX;
  for (int64_t k = nplus - 1; k >= 0; --k) {
    int32_t v = order[nplus - 1 - k];
    uint64_t key = ((uint64_t)(off[v + 1] - off[v]) << 32) | (uint32_t)v;
    sufmin[k] = key < sufmin[k + 1] ? key : sufmin[k + 1];
  }
  {
    int64_t M = -1; /* max cm over neighbours of labels < k */
    int64_t have_prev = 0;
    int64_t prev_p = 0;
    uint64_t prev_key = 0;
    for (int64_t k = 0; k < nplus; ++k) {
      int32_t v = order[nplus - 1 - k];
      uint64_t key = ((uint64_t)(off[v + 1] - off[v]) << 32) | (uint32_t)v;
      int64_t p = INT64_MAX, mx = -1;
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        int64_t c = cm[cols[e]];
        if (c < p) p = c;
        if (c > mx) mx = c;
      }
      if (M < k) {
        if (key != sufmin[k]) { rc = -3; goto done; }
      } else {
        if (p >= k) { rc = -4; goto done; }
        if (have_prev) {
          if (p < prev_p || (p == prev_p && key <= prev_key)) { rc = -5; goto done; }
        }
        have_prev = 1;
        prev_p = p;
        prev_key = key;
      }
      if (mx > M) M = mx;
    }
  }
done:
  free(order);
  free(cm);
  free(sufmin);
  return rc;
}
