/*
 * Densest-subgraph discovery by parallel peeling on one AMD Instinct
 * MI355X (gfx950): C ABI of the peeling part of libkws.so.
 *
 * The operation (the paper's Section 2.1, Equation 1, and the parallel
 * peeling algorithm of Section 4.1, Algorithm 2):
 *
 *   G = (V, E), directed edges e = (src, dst) without self-loops; an edge
 *   is incident to both endpoints. For S a subset of V,
 *     f(S)   = sum_{u in S} a_u + sum_{e in E, src(e), dst(e) in S} c_e,
 *     g(S)   = f(S) / |S|,
 *     w_u(S) = f(S) - f(S \ {u}) (the peeling weight).
 *   Starting from S_0 = V, round i removes every u in S_{i-1} with
 *   w_u(S_{i-1}) <= k (1 + eps) g(S_{i-1}), until nothing is left; the
 *   answer is the first S_i of largest g.
 *
 * The long-tail optimisations of Section 5 (kws_dsd_params.mode):
 *   KWS_DSD_GPO (Algorithm 3): a global threshold tau_max, 0 at first and
 *     raised at the start of every round to g(S_{i-1}) / (k (1 + eps)) when
 *     that is larger; round i removes w_u <= max(tau_max, k (1 + eps) g).
 *   KWS_DSD_LPO (Algorithm 4): as GPO, then, while some u in S_i has
 *     w_u(S_i) < g(S_i), every u with w_u(S_i) < max(tau_max, g(S_i)) is
 *     trimmed from S_i; S_i after its trimming is the round's set (and the
 *     candidate for the densest).
 *
 * Metrics (Section 2.1 and the example listing of Section 3):
 *   KWS_DSD_DG  a = 0, c = 1 (edge density)
 *   KWS_DSD_DW  a = 0, c = the given edge weight
 *   KWS_DSD_FD  a = the given vertex weight, c_e = 1 / ln(deg(src(e)) + 5)
 *               with deg the in- plus out-degree in G, rounded to the
 *               nearest multiple of 2^-24 (weights are integers in 2^-24
 *               units, vertex weights included).
 * All arithmetic is exact integer arithmetic: eps = eps_num / eps_den and
 * ratios are compared by cross-multiplication, so the rounds, the sizes,
 * the f values and the answer are deterministic.
 *
 * Errors: the kws_status codes of kws.h; kws_last_error() describes the
 * last failure of the calling thread.
 */
#ifndef DSD_H
#define DSD_H

#include <stdint.h>

#include "kws.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { KWS_DSD_DG = 0, KWS_DSD_DW = 1, KWS_DSD_FD = 2 };
#define KWS_DSD_ALIVE 0x7fffffff   /* peel round of a vertex never peeled (not returned) */

typedef struct kws_dsd_graph kws_dsd_graph;

/* Host arrays, copied at load (the caller keeps ownership).
 *   src[m], dst[m]  edge endpoints, 0 <= id < n, src != dst; repeated edges
 *                   are separate edges
 *   edge_w[m]       DW edge weights (>= 0, sum below 2^55); NULL for DG and FD
 *   vertex_w[n]     FD vertex weights (>= 0, 2^-24 units); NULL for DG and DW
 *   metric          KWS_DSD_DG, KWS_DSD_DW or KWS_DSD_FD
 * Device memory held by the graph: 4 B per edge endpoint (2m endpoints;
 * DW and FD add 16 B: the weight and a running sum) and about 60 B per
 * vertex; the load itself also takes 16 B per endpoint (32 B for DW and FD)
 * for the sort that orders the rows, freed before it returns.
 * KWS_EINVAL on a malformed graph (nothing is allocated then), KWS_ENOMEM
 * if the device copies do not fit. */
typedef struct {
  int32_t n;
  int64_t m;
  const int32_t *src;
  const int32_t *dst;
  const int64_t *edge_w;
  const int64_t *vertex_w;
  int32_t metric;
} kws_dsd_desc;
kws_status kws_dsd_load(const kws_dsd_desc *d, kws_dsd_graph **out);
void kws_dsd_free(kws_dsd_graph *g);

/* k: 2 for the three metrics (the factor of Theorem 4.2); eps_num in
 * 0..1000, eps_den in 1..1000; k (1 + eps) below 2 is KWS_EINVAL (the
 * mean peeling weight is at most 2 g, so only from 2 on is every round
 * sure to peel a vertex); profile = 1 brackets the kernel classes of
 * profile_classes with HIP events (the summary's *_ms and launches fields;
 * the events are read once the run has finished); mode: see above. */
enum { KWS_DSD_PLAIN = 0, KWS_DSD_GPO = 1, KWS_DSD_LPO = 2 };
typedef struct {
  int32_t k;
  int32_t eps_num;
  int32_t eps_den;
  int32_t profile;
  int32_t mode;          /* KWS_DSD_PLAIN (Algorithm 2), KWS_DSD_GPO or KWS_DSD_LPO */
  int32_t profile_classes;   /* with profile: bit 0 decide, 1 update, 2 reduce; 0 = all */
} kws_dsd_params;

typedef struct {
  int32_t rounds;        /* R: S_R is empty */
  int32_t best;          /* index of the densest S_i */
  int64_t best_size;     /* |S_best| */
  int64_t best_f;        /* f(S_best) */
  int64_t incidences;    /* edge endpoints of the graph (2m) */
  double decide_ms, update_ms, reduce_ms;   /* summed kernel time (profile = 1) */
  int64_t decide_launches, update_launches, reduce_launches;
  int64_t trims;         /* trimming steps (LPO) */
  int64_t steps;         /* rounds + trimming steps */
} kws_dsd_summary;

/* Runs the peeling on the graph's device copy. Outputs (host memory, each
 * may be NULL):
 *   peel_round[n]           the round (1..R) in which each vertex was peeled
 *                           or trimmed;
 *                           S_best = { v : peel_round[v] > best }. With NULL
 *                           the rounds stay in device memory only (see
 *                           kws_dsd_rounds)
 *   sizes[cap], f[cap]      |S_i| and f(S_i) for i = 0..R
 * KWS_EOVERFLOW if R + 1 > cap (with sizes or f given), KWS_EINVAL on bad
 * parameters, KWS_EDEVICE on a device failure. */
kws_status kws_dsd_peel(kws_dsd_graph *g, const kws_dsd_params *p, int32_t *peel_round, int64_t *sizes,
                        int64_t *f, int32_t cap, kws_dsd_summary *summary);

/* The peel rounds of the last finished kws_dsd_peel on g: copied into
 * peel_round[n] (host memory) if it is not NULL, and the address of the
 * library's device array of n int32 (on the device g was loaded on) stored
 * in *device_rounds if that is not NULL. The device array is owned by g and
 * holds these rounds until the next kws_dsd_peel or kws_dsd_free on g.
 * KWS_EINVAL before the first run, KWS_EDEVICE on a device failure. */
kws_status kws_dsd_rounds(kws_dsd_graph *g, int32_t *peel_round, const int32_t **device_rounds);

#ifdef __cplusplus
}
#endif

#endif
