/*
 * TEST INFRASTRUCTURE - the CPU oracle for distance-bounded graph keyword
 * search. Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it. It shares no code with the GPU library.
 *
 * What it computes (the plain definition, written out; one keyword at a
 * time, one thread, no blocking or bit-parallelism):
 *
 *   G = (V, E) directed; out(u) = forward CSR row of u.
 *   S_t = vertices carrying label t, or (with a type tree) carrying any
 *         label whose chain of parents reaches t. Found by walking parents.
 *   dist_t(r) = length of a shortest directed path r -> ... -> v, v in S_t,
 *         if that length is <= d_max; otherwise infinity (255). Computed by
 *         a FIFO breadth-first search over reverse edges from all of S_t,
 *         expanding a vertex only while its distance is below d_max.
 *   roots = { r : dist_t(r) <= d_max for every keyword t of the query }.
 *   score(r) = sum over keywords of dist_t(r); lower ranks higher.
 *   top-k = roots sorted by (score ascending, vertex id ascending), first
 *         min(k, |roots|).
 *   answer edges of root r: for every keyword t, start at x = r and while
 *         dist_t(x) > 0 step to y = the smallest-id out-neighbour of x with
 *         dist_t(y) = dist_t(x) - 1, emitting (x, y); the union over the
 *         keywords, duplicates removed, sorted by (src, dst).
 *   te = sum over keywords of in-degree(x) for every x expanded (dist < d_max):
 *         the reverse edges a plain per-keyword search scans.
 *
 * Citation: the paper fixes only the notation of this search in its
 * preamble (radius d_max, dist, filter, scr, ans_graph_gen, the type-tree
 * relations and the inverted index); no section defines its semantics.
 * The readings above (edge direction, inclusive radius, sum score, the
 * (score, id) tie-break, the min-id answer path, descendants matching a
 * type keyword) are the ones this project adopts.
 *
 * Infinity is 255, so d_max must be <= 254.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define INF 255

typedef struct {
  int32_t n;
  int64_t m;
  int64_t *fptr;   /* forward CSR */
  int32_t *fcol;
  int64_t *rptr;   /* reverse CSR, built here */
  int32_t *rcol;
  int32_t n_labels;
  int64_t *lptr;
  int32_t *lab;
  int32_t *parent; /* NULL: flat labels */
} orc_graph;

void orc_graph_free(orc_graph *g) {
  if (!g) return;
  free(g->fptr); free(g->fcol); free(g->rptr); free(g->rcol);
  free(g->lptr); free(g->lab); free(g->parent); free(g);
}

/* Copies the inputs and builds the reverse adjacency by counting sort.
 * Returns NULL on malformed input or allocation failure. */
orc_graph *orc_graph_new(int32_t n, const int32_t *row_ptr, const int32_t *col,
                         int32_t n_labels, const int32_t *lab_ptr, const int32_t *lab,
                         const int32_t *type_parent) {
  if (n < 0 || row_ptr[0] != 0) return NULL;
  orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
  g->n = n;
  g->m = row_ptr[n];
  g->fptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  g->fcol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->m ? g->m : 1));
  g->rptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  g->rcol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->m ? g->m : 1));
  for (int32_t u = 0; u <= n; u++) g->fptr[u] = row_ptr[u];
  for (int64_t e = 0; e < g->m; e++) {
    if (col[e] < 0 || col[e] >= n) { orc_graph_free(g); return NULL; }
    g->fcol[e] = col[e];
  }
  /* reverse adjacency: p is in rev(x) for every edge p -> x */
  for (int64_t e = 0; e < g->m; e++) g->rptr[g->fcol[e] + 1]++;
  for (int32_t x = 0; x < n; x++) g->rptr[x + 1] += g->rptr[x];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  memcpy(fill, g->rptr, sizeof(int64_t) * ((size_t)n + 1));
  for (int32_t p = 0; p < n; p++)
    for (int64_t e = g->fptr[p]; e < g->fptr[p + 1]; e++)
      g->rcol[fill[g->fcol[e]]++] = p;
  free(fill);
  g->n_labels = n_labels;
  g->lptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  for (int32_t v = 0; v <= n; v++) g->lptr[v] = lab_ptr[v];
  int64_t nl = lab_ptr[n];
  g->lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nl ? nl : 1));
  for (int64_t i = 0; i < nl; i++) {
    if (lab[i] < 0 || lab[i] >= n_labels) { orc_graph_free(g); return NULL; }
    g->lab[i] = lab[i];
  }
  if (type_parent) {
    g->parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_labels ? n_labels : 1));
    memcpy(g->parent, type_parent, sizeof(int32_t) * (size_t)n_labels);
  }
  return g;
}

int64_t orc_graph_m(const orc_graph *g) { return g->m; }

/* 1 if label l is keyword t, or (type tree) t is reached from l by parents */
static int label_matches(const orc_graph *g, int32_t l, int32_t t) {
  if (!g->parent) return l == t;
  for (int32_t x = l, steps = 0; x >= 0 && steps <= g->n_labels; x = g->parent[x], steps++)
    if (x == t) return 1;
  return 0;
}

/* in_set[v] = 1 iff v is in S_t */
void orc_keyword_set(const orc_graph *g, int32_t t, uint8_t *in_set) {
  for (int32_t v = 0; v < g->n; v++) {
    in_set[v] = 0;
    for (int64_t i = g->lptr[v]; i < g->lptr[v + 1]; i++)
      if (label_matches(g, g->lab[i], t)) { in_set[v] = 1; break; }
  }
}

/* Truncated BFS distances to S_t along edge direction (FIFO search over
 * reverse edges). dist[v] in {0..d_max} or INF. Returns the scanned
 * reverse-edge count (in-degrees of the expanded vertices). */
int64_t orc_distances(const orc_graph *g, int32_t t, int32_t d_max, uint8_t *dist) {
  int32_t n = g->n;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  uint8_t *in_set = (uint8_t *)malloc((size_t)(n ? n : 1));
  orc_keyword_set(g, t, in_set);
  int64_t head = 0, tail = 0, te = 0;
  for (int32_t v = 0; v < n; v++) {
    dist[v] = INF;
    if (in_set[v]) { dist[v] = 0; queue[tail++] = v; }
  }
  while (head < tail) {
    int32_t x = queue[head++];
    int32_t l = dist[x];
    if (l >= d_max) continue;
    te += g->rptr[x + 1] - g->rptr[x];
    for (int64_t e = g->rptr[x]; e < g->rptr[x + 1]; e++) {
      int32_t p = g->rcol[e];
      if (dist[p] == INF) { dist[p] = (uint8_t)(l + 1); queue[tail++] = p; }
    }
  }
  free(queue); free(in_set);
  return te;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}
typedef struct { int32_t score, id; } scored;
static int cmp_scored(const void *a, const void *b) {
  const scored *x = (const scored *)a, *y = (const scored *)b;
  if (x->score != y->score) return (x->score > y->score) - (x->score < y->score);
  return (x->id > y->id) - (x->id < y->id);
}
typedef struct { int32_t s, d; } edge;
static int cmp_edge(const void *a, const void *b) {
  const edge *x = (const edge *)a, *y = (const edge *)b;
  if (x->s != y->s) return (x->s > y->s) - (x->s < y->s);
  return (x->d > y->d) - (x->d < y->d);
}

/*
 * One query. kw[n_kw] may repeat ids. Outputs (caller-allocated):
 *   ukw[n_kw]                 unique keywords, ascending   (*n_ukw)
 *   roots[k], scores[k]       (*n_roots) entries, ordered by (score, id)
 *   kw_dist[k * n_kw]         row i = distances of roots[i], ukw order
 *   edge_ptr[k + 1], edge_src/edge_dst[edge_cap]   answer edges per root
 *   te                        scanned reverse edges
 * Returns 0, -1 on bad arguments, -2 if edge_cap is too small.
 */
int orc_search(const orc_graph *g, const int32_t *kw, int32_t n_kw, int32_t d_max, int32_t k,
               int32_t *n_ukw, int32_t *ukw, int32_t *n_roots, int32_t *roots, int32_t *scores,
               uint8_t *kw_dist, int64_t *edge_ptr, int32_t *edge_src, int32_t *edge_dst,
               int64_t edge_cap, int64_t *te) {
  int32_t n = g->n;
  *n_roots = 0; *n_ukw = 0; *te = 0;
  if (n_kw < 1 || d_max < 0 || d_max > 254 || k < 0) return -1;
  for (int32_t i = 0; i < n_kw; i++)
    if (kw[i] < 0 || kw[i] >= g->n_labels) return -1;
  /* 1. sorted unique keywords */
  int32_t *K = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_kw);
  memcpy(K, kw, sizeof(int32_t) * (size_t)n_kw);
  qsort(K, (size_t)n_kw, sizeof(int32_t), cmp_i32);
  int32_t nk = 0;
  for (int32_t i = 0; i < n_kw; i++) if (nk == 0 || K[nk - 1] != K[i]) K[nk++] = K[i];
  *n_ukw = nk;
  memcpy(ukw, K, sizeof(int32_t) * (size_t)nk);
  /* 2-3. per-keyword truncated distances */
  uint8_t *dist = (uint8_t *)malloc((size_t)nk * (size_t)(n ? n : 1));
  for (int32_t j = 0; j < nk; j++) *te += orc_distances(g, K[j], d_max, dist + (size_t)j * n);
  /* 4. root filter and score */
  scored *R = (scored *)malloc(sizeof(scored) * (size_t)(n ? n : 1));
  int64_t nr = 0;
  for (int32_t r = 0; r < n; r++) {
    int ok = 1; int32_t s = 0;
    for (int32_t j = 0; j < nk; j++) {
      uint8_t d = dist[(size_t)j * n + r];
      if (d > d_max) { ok = 0; break; }
      s += d;
    }
    if (ok) { R[nr].score = s; R[nr].id = r; nr++; }
  }
  /* 5. order by (score, id), keep k */
  qsort(R, (size_t)nr, sizeof(scored), cmp_scored);
  int32_t take = (int32_t)(nr < k ? nr : k);
  *n_roots = take;
  for (int32_t i = 0; i < take; i++) {
    roots[i] = R[i].id; scores[i] = R[i].score;
    for (int32_t j = 0; j < nk; j++) kw_dist[(size_t)i * nk + j] = dist[(size_t)j * n + R[i].id];
  }
  /* 6. answer edges: min-id successor walk per keyword, union, sort */
  int rc = 0;
  int64_t out = 0;
  edge *buf = (edge *)malloc(sizeof(edge) * ((size_t)nk * (size_t)(d_max + 1) + 1));
  edge_ptr[0] = 0;
  for (int32_t i = 0; i < take; i++) {
    int64_t cnt = 0;
    for (int32_t j = 0; j < nk; j++) {
      const uint8_t *dj = dist + (size_t)j * n;
      int32_t x = roots[i];
      while (dj[x] > 0) {
        int32_t want = dj[x] - 1, y = -1;
        for (int64_t e = g->fptr[x]; e < g->fptr[x + 1]; e++) {
          int32_t w = g->fcol[e];
          if (dj[w] == want && (y < 0 || w < y)) y = w;
        }
        buf[cnt].s = x; buf[cnt].d = y; cnt++;
        x = y;
      }
    }
    qsort(buf, (size_t)cnt, sizeof(edge), cmp_edge);
    for (int64_t e = 0; e < cnt; e++) {
      if (e > 0 && buf[e].s == buf[e - 1].s && buf[e].d == buf[e - 1].d) continue;
      if (out >= edge_cap) { rc = -2; break; }
      edge_src[out] = buf[e].s; edge_dst[out] = buf[e].d; out++;
    }
    edge_ptr[i + 1] = out;
    if (rc) break;
  }
  free(buf); free(R); free(dist); free(K);
  return rc;
}
