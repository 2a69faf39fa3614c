/*
 * TEST INFRASTRUCTURE - the CPU oracle for parallel peeling (densest
 * subgraph discovery). Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it. It shares no code with the GPU library.
 *
 * What it computes, written out from the definitions (Section 2.1,
 * Equation 1) and the round structure of the parallel peeling algorithm
 * (Section 4.1, Algorithm 2), one thread, every sum recomputed from
 * scratch in every round:
 *
 *   G = (V, E) with directed edges e = (src, dst), no self-loops; an edge
 *   is incident to both of its endpoints.
 *   f(S)   = sum_{u in S} a_u + sum_{e in E, src and dst in S} c_e
 *   g(S)   = f(S) / |S|
 *   w_u(S) = f(S) - f(S \ {u}) = a_u + sum of c_e over the edges e incident
 *            to u whose other endpoint is in S (the peeling weight)
 *   round i = 1, 2, ... while S_{i-1} is not empty:
 *            U = { u in S_{i-1} : w_u(S_{i-1}) <= k (1 + eps) g(S_{i-1}) },
 *            S_i = S_{i-1} \ U
 *   result  the first i in 0..R with the largest g(S_i) over non-empty S_i.
 *
 * orc_peel_opt adds the long-tail optimisations of Section 5: the global
 * peeling threshold (Algorithm 3) and the local trimming loop
 * (Algorithm 4), in the same from-scratch style.
 *
 * Metric weights (Section 2.1 and the example listing of Section 3):
 *   DG  a_u = 0,  c_e = 1
 *   DW  a_u = 0,  c_e = the given edge weight
 *   FD  a_u = the given vertex weight,
 *       c_e = 1 / ln(deg(src(e)) + 5), deg = in- plus out-degree in G,
 *       rounded to the nearest multiple of 2^-24 (stored as an integer).
 * All weights are integers (fixed point for FD), eps = eps_num / eps_den,
 * and every comparison of ratios is done by cross-multiplication in
 * 128-bit integers, so the result is exact.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef unsigned __int128 u128;

#define PEEL_ALIVE 0x7fffffff

/* FD edge weight of an edge whose source has total degree deg. */
int64_t orc_fd_weight(int64_t deg) {
  return llround(16777216.0 / log((double)deg + 5.0));
}

/*
 * Runs the parallel peeling rounds.
 *   n, m, src[m], dst[m]       the graph (no self-loops: returns -1)
 *   c[m], a[n]                 edge and vertex weights (integers >= 0)
 *   k, eps_num, eps_den        threshold k (1 + eps_num / eps_den) g
 *   peel_round[n] (out)        the round in which each vertex is peeled (1-based)
 *   sizes[cap], fs[cap] (out)  |S_i| and f(S_i) for i = 0..rounds
 *   *rounds (out)              R; *best (out) the index of the densest S_i
 * Returns 0, -1 on bad input, -2 if more than cap - 1 rounds would be needed.
 */
int orc_peel(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *c, const int64_t *a,
             int32_t k, int32_t eps_num, int32_t eps_den, int32_t *peel_round, int64_t *sizes, int64_t *fs,
             int32_t cap, int32_t *rounds, int32_t *best) {
  if (n < 0 || m < 0 || k < 1 || eps_num < 0 || eps_den < 1 || cap < 1) return -1;
  /* progress needs k (1 + eps) >= 2: the mean peeling weight is
     (sum a + 2 sum c) / |S| <= 2 g, so the lightest vertex is peeled */
  if ((int64_t)k * (eps_den + eps_num) < 2 * (int64_t)eps_den) return -1;
  for (int64_t e = 0; e < m; e++)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n || src[e] == dst[e] || c[e] < 0) return -1;
  for (int32_t u = 0; u < n; u++)
    if (a[u] < 0) return -1;
  int64_t *w = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!w) return -1;
  for (int32_t u = 0; u < n; u++) peel_round[u] = PEEL_ALIVE;
  int32_t i = 0, alive = n;
  int32_t bi = -1;
  int64_t bf = 0, bs = 1;
  for (;;) {
    /* f(S_i) and |S_i| from the definition */
    int64_t f = 0;
    for (int32_t u = 0; u < n; u++)
      if (peel_round[u] == PEEL_ALIVE) f += a[u];
    for (int64_t e = 0; e < m; e++)
      if (peel_round[src[e]] == PEEL_ALIVE && peel_round[dst[e]] == PEEL_ALIVE) f += c[e];
    sizes[i] = alive;
    fs[i] = f;
    /* densest so far: f / alive > bf / bs, first maximum kept */
    if (alive > 0 && (bi < 0 || (u128)f * (u128)bs > (u128)bf * (u128)alive)) {
      bi = i;
      bf = f;
      bs = alive;
    }
    if (alive == 0) break;
    if (i + 1 >= cap) { free(w); return -2; }
    /* peeling weights w_u(S_i) from the definition */
    for (int32_t u = 0; u < n; u++) w[u] = a[u];
    for (int64_t e = 0; e < m; e++)
      if (peel_round[src[e]] == PEEL_ALIVE && peel_round[dst[e]] == PEEL_ALIVE) {
        w[src[e]] += c[e];
        w[dst[e]] += c[e];
      }
    /* U: w_u * |S| * den <= k * (den + num) * f */
    const u128 rhs = (u128)(uint64_t)k * (u128)(uint64_t)(eps_den + eps_num) * (u128)(uint64_t)f;
    i++;
    int32_t removed = 0;
    for (int32_t u = 0; u < n; u++)   /* w[] was computed for S_{i-1}, before any removal */
      if (peel_round[u] == PEEL_ALIVE && (u128)(uint64_t)w[u] * (u128)(uint64_t)alive * (u128)(uint64_t)eps_den <= rhs) {
        peel_round[u] = i;
        removed++;
      }
    alive -= removed;
    if (removed == 0) { free(w); return -1; }   /* cannot happen for k (1 + eps) >= 2 */
  }
  *rounds = i;
  *best = bi < 0 ? 0 : bi;
  free(w);
  return 0;
}

/*
 * Sequential peeling (Section 2.2, Algorithm 1): remove one vertex of
 * smallest peeling weight at a time (smallest id among equals) and keep the
 * first densest S_i. in_best[n] (out) marks the returned set; *bf, *bs its
 * f and size. Only for small graphs (O(n (n + m))).
 */
int orc_peel_sequential(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *c,
                        const int64_t *a, uint8_t *in_best, int64_t *bf_out, int64_t *bs_out) {
  uint8_t *alive = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t *w = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!alive || !order || !w) { free(alive); free(order); free(w); return -1; }
  for (int32_t u = 0; u < n; u++) alive[u] = 1;
  int64_t bf = 0, bs = 1;
  int32_t best_removed = -1;   /* number of removals before the best set */
  for (int32_t r = 0; r <= n; r++) {
    const int32_t size = n - r;
    int64_t f = 0;
    for (int32_t u = 0; u < n; u++)
      if (alive[u]) f += a[u];
    for (int64_t e = 0; e < m; e++)
      if (alive[src[e]] && alive[dst[e]]) f += c[e];
    if (size > 0 && (best_removed < 0 || (u128)f * (u128)bs > (u128)bf * (u128)size)) {
      best_removed = r;
      bf = f;
      bs = size;
    }
    if (size == 0) break;
    for (int32_t u = 0; u < n; u++) w[u] = a[u];
    for (int64_t e = 0; e < m; e++)
      if (alive[src[e]] && alive[dst[e]]) { w[src[e]] += c[e]; w[dst[e]] += c[e]; }
    int32_t pick = -1;
    for (int32_t u = 0; u < n; u++)
      if (alive[u] && (pick < 0 || w[u] < w[pick])) pick = u;
    alive[pick] = 0;
    order[r] = pick;
  }
  for (int32_t u = 0; u < n; u++) in_best[u] = 1;
  for (int32_t r = 0; r < best_removed; r++) in_best[order[r]] = 0;
  *bf_out = bf;
  *bs_out = bs;
  free(alive); free(order); free(w);
  return 0;
}

/* f(S) and the peeling weights w_u(S) of every u in S, from the definitions;
 * S = { u : peel_round[u] == PEEL_ALIVE }. */
static int64_t opt_weights(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *c,
                           const int64_t *a, const int32_t *peel_round, int64_t *w) {
  int64_t f = 0;
  for (int32_t u = 0; u < n; u++) {
    w[u] = a[u];
    if (peel_round[u] == PEEL_ALIVE) f += a[u];
  }
  for (int64_t e = 0; e < m; e++)
    if (peel_round[src[e]] == PEEL_ALIVE && peel_round[dst[e]] == PEEL_ALIVE) {
      f += c[e];
      w[src[e]] += c[e];
      w[dst[e]] += c[e];
    }
  return f;
}

/*
 * Peeling with the long-tail optimisations of Section 5. mode 1 is the
 * global peeling threshold of Algorithm 3 (GPO), mode 2 adds the local
 * trimming loop of Algorithm 4 (LPO); mode 0 is Algorithm 2 (as orc_peel).
 * tau_max starts at 0. Outer iteration i, with S = S_{i-1}:
 *   modes 1, 2: tau_max = max(tau_max, g(S) / (k (1 + eps)))
 *   U1 = { u in S : w_u(S) <= max(tau_max, k (1 + eps) g(S)) },  S = S \ U1
 *   mode 2: while some u in S has w_u(S) < g(S):
 *             U2 = { u in S : w_u(S) < max(tau_max, g(S)) },  S = S \ U2
 *   S_i = S; every vertex removed in iteration i (by U1 or a U2) gets peel
 *   round i.
 * The result is the first i in 0..R with the largest g(S_i) over non-empty
 * S_i (S_i after its trimming). tau_max is kept as a fraction A / B and
 * every comparison is cross-multiplied in 128 bits. Outputs as orc_peel,
 * plus *trims (the number of trimming steps). Returns 0, -1 on bad input,
 * -2 if more than cap - 1 iterations would be needed.
 */
int orc_peel_opt(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *c, const int64_t *a,
                 int32_t k, int32_t eps_num, int32_t eps_den, int32_t mode, int32_t *peel_round, int64_t *sizes,
                 int64_t *fs, int32_t cap, int32_t *rounds, int32_t *best, int32_t *trims) {
  if (n < 0 || m < 0 || k < 1 || eps_num < 0 || eps_den < 1 || cap < 1 || mode < 0 || mode > 2) return -1;
  if ((int64_t)k * (eps_den + eps_num) < 2 * (int64_t)eps_den) return -1;   /* as in orc_peel */
  for (int64_t e = 0; e < m; e++)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n || src[e] == dst[e] || c[e] < 0) return -1;
  for (int32_t u = 0; u < n; u++)
    if (a[u] < 0) return -1;
  int64_t *w = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!w) return -1;
  for (int32_t u = 0; u < n; u++) peel_round[u] = PEEL_ALIVE;
  const u128 K1 = (u128)(uint64_t)k * (u128)(uint64_t)(eps_den + eps_num);   /* k (1 + eps) = K1 / den */
  const u128 den = (u128)(uint64_t)eps_den;
  u128 tA = 0, tB = 1;                       /* tau_max = tA / tB */
  int32_t i = 0, alive = n, ntrim = 0;
  int32_t bi = -1;
  int64_t bf = 0, bs = 1;
  int64_t f = opt_weights(n, m, src, dst, c, a, peel_round, w);
  sizes[0] = alive;
  fs[0] = f;
  for (;;) {
    /* S_i is final here: candidate for the densest set */
    if (alive > 0 && (bi < 0 || (u128)f * (u128)bs > (u128)bf * (u128)alive)) {
      bi = i;
      bf = f;
      bs = alive;
    }
    if (alive == 0) break;
    if (i + 1 >= cap) { free(w); return -2; }
    i++;
    /* S = S_{i-1}, weights w = w(S_{i-1}) */
    const u128 s = (u128)(uint64_t)alive;
    if (mode >= 1) {                         /* tau_max = max(tau_max, g / (k (1 + eps))) */
      const u128 nA = (u128)(uint64_t)f * den, nB = s * K1;
      if (nA * tB > tA * nB) { tA = nA; tB = nB; }
    }
    int32_t removed = 0;
    for (int32_t u = 0; u < n; u++) {
      if (peel_round[u] != PEEL_ALIVE) continue;
      const u128 wu = (u128)(uint64_t)w[u];
      const int le_tau = wu * tB <= tA;                                   /* w <= tau_max */
      const int le_g = wu * s * den <= K1 * (u128)(uint64_t)f;           /* w <= k (1 + eps) g */
      if (le_tau || le_g) { peel_round[u] = i; removed++; }
    }
    alive -= removed;
    if (removed == 0) { free(w); return -1; }   /* cannot happen for k (1 + eps) >= 2 */
    f = opt_weights(n, m, src, dst, c, a, peel_round, w);
    if (mode == 2) {
      for (;;) {
        const u128 s2 = (u128)(uint64_t)alive;
        int any = 0;                           /* some u with w_u < g(S) */
        for (int32_t u = 0; u < n && !any; u++)
          if (peel_round[u] == PEEL_ALIVE && (u128)(uint64_t)w[u] * s2 < (u128)(uint64_t)f) any = 1;
        if (!any) break;
        int32_t cut = 0;
        for (int32_t u = 0; u < n; u++) {      /* w_u(S) < max(tau_max, g(S)), from w of this S */
          if (peel_round[u] != PEEL_ALIVE) continue;
          const u128 wu = (u128)(uint64_t)w[u];
          if (wu * tB < tA || wu * s2 < (u128)(uint64_t)f) { peel_round[u] = i; cut++; }
        }
        alive -= cut;
        ntrim++;
        f = opt_weights(n, m, src, dst, c, a, peel_round, w);
      }
    }
    sizes[i] = alive;
    fs[i] = f;
  }
  *rounds = i;
  *best = bi < 0 ? 0 : bi;
  *trims = ntrim;
  free(w);
  return 0;
}
