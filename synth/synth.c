/*
 * Seeded synthetic inputs for the keyword-search workloads: directed graphs
 * (R-MAT, Chung-Lu), Zipf vertex labels, a complete type tree, query sets
 * and Poisson arrival times.
 *
 * This module computes nothing of the search itself (no distances, no
 * scores, no ranking). Both the CPU oracle's tests and the GPU library's
 * tests and benchmark draw their inputs from here.
 *
 * Randomness: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used in counter mode: the
 * i-th number of a stream is the SplitMix64 finaliser applied to
 * key + (i+1) * 0x9E3779B97F4A7C15, where key is derived from
 * (seed, stream id). Every draw is therefore a pure function of
 * (seed, stream, counter); results do not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

/* stream ids: keep every draw site on its own stream */
enum {
  ST_RMAT = 1, ST_VPERM = 2, ST_CL_OUTPERM = 3, ST_CL_INPERM = 4, ST_CL_EDGE = 5,
  ST_LAB_COUNT = 6, ST_LAB_DRAW = 7, ST_LAB_PERM = 8, ST_TREE_PERM = 9,
  ST_Q_SIZE = 10, ST_Q_KW = 11, ST_Q_DMAX = 12, ST_Q_DEPTH = 13, ST_ARRIVAL = 14,
  ST_PERM_GENERIC = 15
};

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t sm_key(uint64_t seed, uint64_t stream) {
  return sm_mix(seed ^ sm_mix(stream * GOLDEN + 0x632BE59BD9B4E019ULL));
}
static inline uint64_t sm_at(uint64_t key, uint64_t ctr) {
  return sm_mix(key + (ctr + 1) * GOLDEN);
}
/* uniform double in [0,1) with 53 random bits */
static inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
/* uniform integer in [0, span) (span < 2^32; the bias is below 2^-32) */
static inline uint64_t below(uint64_t r, uint64_t span) {
  return (uint64_t)(((unsigned __int128)(r >> 32) * span) >> 32);
}

uint64_t syn_key(uint64_t seed, uint64_t stream) { return sm_key(seed, stream); }

uint64_t syn_u64(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return sm_at(sm_key(seed, stream), ctr);
}

/* out[i] = a uniform integer in [lo, hi] from draw i of (seed, stream),
 * by multiply-shift of the 64-bit draw (bias below 2^-40 for ranges under
 * 2^24). */
void syn_uniform_i64(uint64_t seed, uint64_t stream, int64_t count, int64_t lo, int64_t hi, int64_t *out) {
  const uint64_t key = sm_key(seed, stream);
  const unsigned __int128 span = (unsigned __int128)(uint64_t)(hi - lo) + 1u;
  for (int64_t i = 0; i < count; i++)
    out[i] = lo + (int64_t)(((unsigned __int128)sm_at(key, (uint64_t)i) * span) >> 64);
}

/* Fisher-Yates shuffle of 0..n-1, draws from (seed, stream). */
static void make_perm(int64_t n, uint64_t seed, uint64_t stream, int32_t *perm) {
  uint64_t key = sm_key(seed, stream);
  for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; i--) {
    int64_t j = (int64_t)below(sm_at(key, (uint64_t)i), (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

void syn_permutation(int64_t n, uint64_t seed, uint64_t stream, int32_t *perm) {
  make_perm(n, seed, stream, perm);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static void sort_i32(int32_t *a, int64_t len) {
  if (len < 2) return;
  if (len < 24) {
    for (int64_t i = 1; i < len; i++) {
      int32_t v = a[i]; int64_t j = i - 1;
      while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; j--; }
      a[j + 1] = v;
    }
    return;
  }
  qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
}

/*
 * Shared back end: per-row sort, drop self-loops and duplicates, compact.
 * tmp_ptr[n+1] / tmp_col hold the raw rows; writes row_ptr[n+1] and col[],
 * returns the final edge count.
 */
static int64_t clean_rows(int32_t n, const int64_t *tmp_ptr, int32_t *tmp_col,
                          int32_t *row_ptr, int32_t *col) {
  int32_t *newdeg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  #pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t u = 0; u < n; u++) {
    int32_t *r = tmp_col + tmp_ptr[u];
    int64_t len = tmp_ptr[u + 1] - tmp_ptr[u];
    sort_i32(r, len);
    int64_t w = 0;
    for (int64_t i = 0; i < len; i++) {
      if (r[i] == u) continue;
      if (w > 0 && r[w - 1] == r[i]) continue;
      r[w++] = r[i];
    }
    newdeg[u] = (int32_t)w;
  }
  int64_t acc = 0;
  row_ptr[0] = 0;
  for (int32_t u = 0; u < n; u++) { acc += newdeg[u]; row_ptr[u + 1] = (int32_t)acc; }
  #pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t u = 0; u < n; u++)
    memcpy(col + row_ptr[u], tmp_col + tmp_ptr[u], sizeof(int32_t) * (size_t)newdeg[u]);
  free(newdeg);
  return acc;
}

static inline void rmat_sample(uint64_t key, uint64_t i, int scale, double a, double ab,
                               double abc, int32_t *u_out, int32_t *v_out) {
  uint32_t u = 0, v = 0;
  for (int l = 0; l < scale; l++) {
    double r = u01(sm_at(key, i * (uint64_t)scale + (uint64_t)l));
    uint32_t bu, bv;
    if (r < a) { bu = 0; bv = 0; }
    else if (r < ab) { bu = 0; bv = 1; }
    else if (r < abc) { bu = 1; bv = 0; }
    else { bu = 1; bv = 1; }
    u = (u << 1) | bu; v = (v << 1) | bv;
  }
  *u_out = (int32_t)u; *v_out = (int32_t)v;
}

/* Parallel LSD radix sort of 64-bit keys on their low `bits` bits, 11 bits
 * per pass; the result ends up in keys[]. */
static void radix_sort_u64(uint64_t *keys, uint64_t *tmp, int64_t len, int bits) {
  enum { RB = 11, NB = 1 << RB };
  int nth = 1;
  #pragma omp parallel
  {
    #pragma omp single
    nth = omp_get_num_threads();
  }
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)nth * NB);
  uint64_t *src = keys, *dst = tmp;
  int passes = (bits + RB - 1) / RB;
  for (int p = 0; p < passes; p++) {
    const int shift = p * RB;
    memset(cnt, 0, sizeof(int64_t) * (size_t)nth * NB);
    #pragma omp parallel num_threads(nth)
    {
      const int t = omp_get_thread_num();
      const int64_t lo = len * t / nth, hi = len * (t + 1) / nth;
      int64_t *c = cnt + (size_t)t * NB;
      for (int64_t i = lo; i < hi; i++) c[(src[i] >> shift) & (NB - 1)]++;
      #pragma omp barrier
      #pragma omp single
      {
        int64_t acc = 0;
        for (int d = 0; d < NB; d++)
          for (int u = 0; u < nth; u++) {
            int64_t x = cnt[(size_t)u * NB + d];
            cnt[(size_t)u * NB + d] = acc;
            acc += x;
          }
      }
      for (int64_t i = lo; i < hi; i++) dst[c[(src[i] >> shift) & (NB - 1)]++] = src[i];
    }
    uint64_t *x = src; src = dst; dst = x;
  }
  if (src != keys) memcpy(keys, src, sizeof(uint64_t) * (size_t)len);
  free(cnt);
}

/*
 * R-MAT(a,b,c,d=1-a-b-c) with 2^scale vertices and n_samples sampled edges
 * (Chakrabarti, Zhan and Faloutsos, SDM 2004), no noise. Vertex ids are
 * relabelled by a seeded random permutation (Graph500 practice), then
 * self-loops and duplicate edges are dropped. Output is a forward CSR with
 * ascending neighbour ids per row. col must hold n_samples entries.
 * Returns the final edge count m, or -1 on allocation failure.
 */
int64_t syn_rmat_csr(int32_t scale, int64_t n_samples, double a, double b, double c,
                     uint64_t seed, int32_t *row_ptr, int32_t *col) {
  int32_t n = (int32_t)1 << scale;
  uint64_t key = sm_key(seed, ST_RMAT);
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_samples > 0 ? n_samples : 1));
  uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_samples > 0 ? n_samples : 1));
  if (!perm || !keys || !tmp) { free(perm); free(keys); free(tmp); return -1; }
  make_perm(n, seed, ST_VPERM, perm);
  double ab = a + b, abc = a + b + c;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_samples; i++) {
    int32_t u, v;
    rmat_sample(key, (uint64_t)i, scale, a, ab, abc, &u, &v);
    keys[i] = ((uint64_t)(uint32_t)perm[u] << scale) | (uint64_t)(uint32_t)perm[v];
  }
  radix_sort_u64(keys, tmp, n_samples, 2 * scale);
  free(tmp);
  /* sorted by (u, v): drop self-loops and repeats while filling the CSR */
  const uint64_t vmask = ((uint64_t)1 << scale) - 1;
  int64_t m = 0, e = 0;
  row_ptr[0] = 0;
  for (int32_t u = 0; u < n; u++) {
    while (e < n_samples && (int32_t)(keys[e] >> scale) == u) {
      const uint64_t k = keys[e];
      const int32_t v = (int32_t)(k & vmask);
      if (v != u && (e == 0 || keys[e - 1] != k)) col[m++] = v;
      e++;
    }
    row_ptr[u + 1] = (int32_t)m;
  }
  free(perm); free(keys);
  return m;
}

/* ---- open-addressing set of 64-bit keys (for Chung-Lu distinct edges) ---- */
typedef struct { uint64_t *slot; uint64_t mask; } u64set;
static int set_insert(u64set *s, uint64_t k) {  /* 1 if new */
  uint64_t h = sm_mix(k) & s->mask;
  for (;;) {
    uint64_t x = s->slot[h];
    if (x == UINT64_MAX) { s->slot[h] = k; return 1; }
    if (x == k) return 0;
    h = (h + 1) & s->mask;
  }
}

static int64_t lower_bound_d(const double *cdf, int64_t len, double x) {
  int64_t lo = 0, hi = len;              /* first index with cdf[i] > x */
  while (lo < hi) { int64_t mid = (lo + hi) >> 1; if (cdf[mid] > x) hi = mid; else lo = mid + 1; }
  return lo < len ? lo : len - 1;
}

/*
 * Chung-Lu directed graph: out- and in-weights w_i = (i+1)^(-1/(gamma-1)),
 * each assigned to vertices through its own seeded permutation. Edges
 * (u,v) are drawn with probability proportional to w_out(u) * w_in(v)
 * until exactly m distinct non-loop edges exist. col must hold m entries.
 * Returns m, or -1 if the pair space is too small.
 */
int64_t syn_chung_lu_csr(int32_t n, int64_t m, double gamma, uint64_t seed,
                         int32_t *row_ptr, int32_t *col) {
  if ((double)m > 0.5 * (double)n * (double)(n - 1)) return -1;
  double *cdf = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t *pout = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *pin = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  double acc = 0.0, ex = -1.0 / (gamma - 1.0);
  for (int32_t i = 0; i < n; i++) { acc += pow((double)(i + 1), ex); cdf[i] = acc; }
  make_perm(n, seed, ST_CL_OUTPERM, pout);
  make_perm(n, seed, ST_CL_INPERM, pin);
  uint64_t cap = 1; while (cap < (uint64_t)m * 4) cap <<= 1;
  u64set s; s.mask = cap - 1; s.slot = (uint64_t *)malloc(sizeof(uint64_t) * cap);
  memset(s.slot, 0xFF, sizeof(uint64_t) * cap);
  int32_t *eu = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  uint64_t key = sm_key(seed, ST_CL_EDGE);
  int64_t got = 0; uint64_t ctr = 0;
  while (got < m) {
    int32_t u = pout[lower_bound_d(cdf, n, u01(sm_at(key, ctr)) * acc)];
    int32_t v = pin[lower_bound_d(cdf, n, u01(sm_at(key, ctr + 1)) * acc)];
    ctr += 2;
    if (u == v) continue;
    if (!set_insert(&s, (uint64_t)u * (uint64_t)n + (uint64_t)v)) continue;
    eu[got] = u; ev[got] = v; got++;
  }
  int64_t *ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t i = 0; i < m; i++) ptr[eu[i] + 1]++;
  for (int32_t u = 0; u < n; u++) ptr[u + 1] += ptr[u];
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  memcpy(cur, ptr, sizeof(int64_t) * (size_t)n);
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  for (int64_t i = 0; i < m; i++) tmp[cur[eu[i]]++] = ev[i];
  int64_t mm = clean_rows(n, ptr, tmp, row_ptr, col);
  free(cdf); free(pout); free(pin); free(s.slot); free(eu); free(ev); free(ptr); free(cur); free(tmp);
  return mm;
}

/* Zipf(s) cumulative weights over ranks 1..L: cdf[r-1] = sum_{i<=r} i^-s */
static double *zipf_cdf(int32_t L, double s) {
  double *cdf = (double *)malloc(sizeof(double) * (size_t)L);
  double acc = 0.0;
  for (int32_t r = 0; r < L; r++) { acc += pow((double)(r + 1), -s); cdf[r] = acc; }
  return cdf;
}

/*
 * Vertex labels: each vertex gets a count uniform on [lo, hi], then that
 * many distinct values drawn by Zipf(s) rank (inverse-CDF sampling) and
 * mapped through a seeded permutation of 0..L-1 (the "label permutation",
 * stream ST_LAB_PERM of this seed; syn_queries reuses it so that popular
 * keywords are popular labels). Labels of a vertex are sorted ascending.
 * lab must hold n*hi entries; returns the total label count.
 */
int64_t syn_labels_zipf(int32_t n, int32_t L, double s, int32_t lo, int32_t hi, uint64_t seed,
                        int32_t *lab_ptr, int32_t *lab) {
  if (L < hi || lo < 0 || hi < lo) return -1;
  double *cdf = zipf_cdf(L, s);
  double tot = cdf[L - 1];
  int32_t *lperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
  make_perm(L, seed, ST_LAB_PERM, lperm);
  uint64_t kc = sm_key(seed, ST_LAB_COUNT), kd = sm_key(seed, ST_LAB_DRAW);
  lab_ptr[0] = 0;
  for (int32_t v = 0; v < n; v++)
    lab_ptr[v + 1] = lab_ptr[v] + lo + (int32_t)below(sm_at(kc, (uint64_t)v), (uint64_t)(hi - lo + 1));
  #pragma omp parallel for schedule(static)
  for (int32_t v = 0; v < n; v++) {
    int32_t *out = lab + lab_ptr[v];
    int32_t cnt = lab_ptr[v + 1] - lab_ptr[v], got = 0;
    for (uint64_t j = 0; got < cnt; j++) {
      int32_t x = lperm[lower_bound_d(cdf, L, u01(sm_at(kd, (uint64_t)v * 1024 + j)) * tot)];
      int dup = 0;
      for (int32_t i = 0; i < got; i++) dup |= (out[i] == x);
      if (!dup) out[got++] = x;
    }
    sort_i32(out, cnt);
  }
  free(cdf); free(lperm);
  return lab_ptr[n];
}

/*
 * Complete fanout-ary type tree: root at depth 0, leaves at depth `depth`.
 * Nodes are numbered in BFS order and then renamed by a seeded permutation,
 * so type ids carry no structure. parent[t] = parent type id, -1 for the
 * root. leaves[] receives the leaf type ids (BFS order of the leaves,
 * renamed). Returns the number of types; n_leaves_out gets the leaf count.
 */
int64_t syn_type_tree(int32_t fanout, int32_t depth, uint64_t seed, int32_t *parent,
                      int32_t *leaves, int64_t *n_leaves_out) {
  int64_t total = 0, lvl = 1, first_leaf = 0;
  for (int32_t d = 0; d <= depth; d++) { if (d == depth) first_leaf = total; total += lvl; lvl *= fanout; }
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
  make_perm(total, seed, ST_TREE_PERM, perm);
  for (int64_t i = 0; i < total; i++)
    parent[perm[i]] = i == 0 ? -1 : perm[(i - 1) / fanout];
  for (int64_t i = first_leaf; i < total; i++) leaves[i - first_leaf] = perm[i];
  *n_leaves_out = total - first_leaf;
  free(perm);
  return total;
}

/*
 * Query sets. Query q has n_kw[q] distinct keywords, n_kw uniform on
 * [mq_lo, mq_hi]; each keyword is a Zipf(s) rank over L labels mapped
 * through the label permutation of label_seed (the same map used by
 * syn_labels_zipf). d_max[q] is drawn uniformly from dmax_set[0..n_dmax).
 * kw is [nq * mq_hi], row q holds n_kw[q] valid entries.
 *
 * Hierarchical variant (leaf_ids != NULL): the Zipf draw picks a leaf
 * (through leaf_ids after the permutation) and the keyword is that leaf's
 * ancestor at a depth uniform on [hd_lo, hd_hi] (leaves sit at depth
 * leaf_depth; parent[] gives the tree).
 */
int32_t syn_queries(int32_t nq, int32_t L, double s, int32_t mq_lo, int32_t mq_hi,
                    const int32_t *dmax_set, int32_t n_dmax, uint64_t label_seed, uint64_t seed,
                    const int32_t *leaf_ids, const int32_t *parent, int32_t leaf_depth,
                    int32_t hd_lo, int32_t hd_hi,
                    int32_t *kw, int32_t *n_kw, int32_t *d_max) {
  if (L < mq_hi || mq_lo < 1 || mq_hi < mq_lo || n_dmax < 1) return -1;
  double *cdf = zipf_cdf(L, s);
  double tot = cdf[L - 1];
  int32_t *lperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
  make_perm(L, label_seed, ST_LAB_PERM, lperm);
  uint64_t ks = sm_key(seed, ST_Q_SIZE), kk = sm_key(seed, ST_Q_KW);
  uint64_t kd = sm_key(seed, ST_Q_DMAX), kh = sm_key(seed, ST_Q_DEPTH);
  for (int32_t q = 0; q < nq; q++) {
    int32_t cnt = mq_lo + (int32_t)below(sm_at(ks, (uint64_t)q), (uint64_t)(mq_hi - mq_lo + 1));
    int32_t *out = kw + (int64_t)q * mq_hi, got = 0;
    for (uint64_t j = 0; got < cnt && j < 1000000; j++) {
      uint64_t c = (uint64_t)q * 1000000ULL + j;
      int32_t x = lperm[lower_bound_d(cdf, L, u01(sm_at(kk, c)) * tot)];
      if (leaf_ids) {
        x = leaf_ids[x];
        int32_t want = hd_lo + (int32_t)below(sm_at(kh, c), (uint64_t)(hd_hi - hd_lo + 1));
        for (int32_t d = leaf_depth; d > want; d--) x = parent[x];
      }
      int dup = 0;
      for (int32_t i = 0; i < got; i++) dup |= (out[i] == x);
      if (!dup) out[got++] = x;
    }
    n_kw[q] = got;
    d_max[q] = dmax_set[below(sm_at(kd, (uint64_t)q), (uint64_t)n_dmax)];
  }
  free(cdf); free(lperm);
  return 0;
}

/* Poisson process of rate lam: t[0] is the first arrival, gaps Exp(lam). */
void syn_arrivals(int64_t count, double lam, uint64_t seed, double *t) {
  uint64_t key = sm_key(seed, ST_ARRIVAL);
  double acc = 0.0;
  for (int64_t i = 0; i < count; i++) {
    acc += -log1p(-u01(sm_at(key, (uint64_t)i))) / lam;
    t[i] = acc;
  }
}
