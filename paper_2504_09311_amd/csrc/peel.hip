// Densest-subgraph discovery by parallel peeling (the paper's Section 4.1,
// Algorithm 2), with the DG, DW and FD weight functions of Section 2.1.
//
// Layout: vertices are renumbered at load by descending initial peeling
// weight (ties by id), so the first round's survivors are the smallest ids
// and the later rounds' survivors, the dense part, stay among them; every
// edge is stored twice in an incidence CSR (once in the row of each
// endpoint, rows sorted by neighbour id) with its weight and a running sum
// of the weights; per vertex the current peeling weight w (int64), the
// round it was peeled in (copied out in the caller's ids at the end of a
// run) and an alive bit (the bitmap is n/8 bytes, so random alive tests
// hit L2), and two ping-pong lists of the vertices still alive. Decide also
// records one more than the largest surviving id: neighbours at or above
// it are gone without a test, and when the survivors are exactly the ids
// below it the bitmap is not read at all. A step is four kinds of launch
// (plus one thread that picks its kind), all on the device:
//   decide  scan the alive list: w_u * |S| * den <= k * (den + num) * f
//           (128-bit products) puts u on the peeled list, else on the next
//           alive list; appends are aggregated per block;
//   update  push: the peeled vertices subtract their edge weights from the
//           neighbours still alive (64-bit atomics); or pull: the survivors
//           re-sum their alive neighbours (a binary search per survivor,
//           or a wavefront per row piece); push only while the peeled
//           vertices have a small share of the work, as it pays an atomic
//           per alive neighbour (chosen on the device);
//   reduce  sum of a + w over the survivors (= 2 f(S_i));
//   end     one thread: f, |S|, the per-round record and the densest S_i.
// The host only enqueues steps and reads |S| every few steps to stop.
// Everything is integer arithmetic, so results do not depend on the order
// of the atomics.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "dsd.h"
#include "kws_internal.h"

namespace kws {
namespace {

typedef unsigned __int128 u128;
constexpr int32_t ALIVE = KWS_DSD_ALIVE;
constexpr int SMALL_DEG = 64;   // rows above this are summed by a wavefront at start
constexpr int SMALL_PUSH = 16;  // peeled rows up to this are pushed by one thread
constexpr int PIECE = 1024;     // incidences of a survivor's row summed by one wavefront (pull)
constexpr uint32_t FEW_PIECES = 4;   // rows of more pieces are listed by the whole wavefront
constexpr int MAX_CUTS = 64;          // steps whose survivor bounds are kept for the export
// push costs an atomic per alive neighbour, pull streams ids and tests a bit:
// push is taken while the removed vertices have at most 1/PUSH_COST of the
// survivors' incidences
constexpr unsigned long long PUSH_COST = 16;

// Kinds of step: a peeling step opens a round (Algorithm 2's test, or the
// thresholds of Algorithms 3 and 4); a trimming step (Algorithm 4) removes
// the vertices lighter than max(tau_max, g(S)) inside the round; after the
// set is empty every step does nothing.
enum { STEP_PEEL = 0, STEP_TRIM = 1, STEP_DONE = 2 };
enum { MODE_PLAIN = 0, MODE_GPO = 1, MODE_LPO = 2 };

// Every counter that blocks add to atomically has a 128-byte line of its
// own: atomics on one line are serialised, on separate lines they proceed
// in parallel.
struct PeelScalars {
  alignas(128) unsigned long long cnt[2];   // lengths of the two alive lists
  alignas(128) unsigned long long nu;       // vertices removed by the current step with small rows
  alignas(128) unsigned long long nu_big;   // ... with rows above SMALL_PUSH incidences (listed from the end)
  alignas(128) unsigned long long sum2;     // sum of a + w over the survivors
  alignas(128) unsigned long long deg_peel; // incidences of the vertices removed by the current step
  alignas(128) unsigned long long deg_keep; // incidences of the survivors
  alignas(128) unsigned long long nlt;      // survivors with w_u < g(S) (trimming test)
  alignas(128) unsigned long long nitems;   // pull work items (row pieces of the survivors)
  alignas(128) int bound;                   // 1 + the largest id among the survivors of the current step
  alignas(128) unsigned long long trims;    // trimming steps so far
  unsigned long long tau_lo, tau_hi, tau_den;   // tau_max = (tau_hi:tau_lo) / tau_den
  long long f, s;              // f(S), |S| of the current set
  long long best_f, best_s;
  int best_i, round, phase;
  // the survivors after step i were the ids below cut[i] (i < MAX_CUTS),
  // as long as every step so far left such a prefix (not nonprefix)
  int ncut, nonprefix;
  int cut[MAX_CUTS], cut_round[MAX_CUTS];
};

// incidence keys of the relabelled graph, (row << 32) | neighbour, one
// from each end of every edge, with the edge weight as value: sorted, they
// give every row in order of neighbour id
__global__ __launch_bounds__(BLOCK) void k_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                                                const int64_t *__restrict__ ew, int64_t m, int metric,
                                                const int64_t *__restrict__ fd_table,
                                                const int32_t *__restrict__ deg, const int32_t *__restrict__ inv,
                                                unsigned long long *__restrict__ keys, int64_t *__restrict__ vals) {
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < m; e += (int64_t)gridDim.x * BLOCK) {
    const int32_t u = inv[src[e]], v = inv[dst[e]];
    keys[2 * e] = ((unsigned long long)u << 32) | (uint32_t)v;
    keys[2 * e + 1] = ((unsigned long long)v << 32) | (uint32_t)u;
    if (vals) {
      const int64_t c = metric == KWS_DSD_DW ? ew[e] : fd_table[deg[u]];   // FD: by the source's degree
      vals[2 * e] = c;
      vals[2 * e + 1] = c;
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_unpack(const unsigned long long *__restrict__ keys, int64_t count,
                                                  int32_t *__restrict__ nbr) {
  for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < count; j += (int64_t)gridDim.x * BLOCK)
    nbr[j] = (int32_t)(uint32_t)keys[j];
}

// initial peeling weights: a_u plus the weights of all incident edges
// Peeling weights of the whole graph, w_u(V) = a_u + sum of the incident
// edge weights; computed once at load (rows above SMALL_DEG are finished by
// k_w0_big).
__global__ __launch_bounds__(BLOCK) void k_w0_small(int32_t n, const int64_t *__restrict__ ptr,
                                                    const int64_t *__restrict__ wt, const int64_t *__restrict__ a,
                                                    int64_t *__restrict__ w0) {
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
    const int64_t b = ptr[v], e = ptr[v + 1];
    int64_t s = a ? a[v] : 0;
    if (!wt) s += e - b;
    else if (e - b <= SMALL_DEG)
      for (int64_t j = b; j < e; j++) s += wt[j];
    w0[v] = s;
  }
}

// start of a run: S_0 = V (the first step reads its alive list as the
// identity, so none is written)
__global__ __launch_bounds__(BLOCK) void k_start(int32_t n, const int64_t *__restrict__ w0, int64_t *__restrict__ w,
                                                 int32_t *__restrict__ rnd_in, uint32_t *__restrict__ alive) {
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
    w[v] = w0[v];
    rnd_in[v] = ALIVE;
    if ((v & 31) == 0) alive[v >> 5] = n - v >= 32 ? ~0u : (1u << (n - v)) - 1u;
  }
}

__global__ __launch_bounds__(BLOCK) void k_w0_big(const int32_t *__restrict__ big, int32_t nbig,
                                                    const int64_t *__restrict__ ptr, const int64_t *__restrict__ wt,
                                                    int64_t *__restrict__ w) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6; i < nbig;
       i += ((int64_t)gridDim.x * BLOCK) >> 6) {
    const int32_t v = big[i];
    unsigned long long s = 0;
    for (int64_t j = ptr[v] + lane; j < ptr[v + 1]; j += 64) s += (unsigned long long)wt[j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) w[v] += (int64_t)s;
  }
}

// 2 f(V) = sum of a + w over V, once at load
__global__ __launch_bounds__(BLOCK) void k_sum_all(int32_t n, const int64_t *__restrict__ a,
                                                   const int64_t *__restrict__ w0, unsigned long long *out) {
  __shared__ unsigned long long s_part[BLOCK / 64];
  unsigned long long t = 0;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK)
    t += (unsigned long long)w0[v] + (a ? (unsigned long long)a[v] : 0ull);
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long u = 0;
    for (int i = 0; i < BLOCK / 64; i++) u += s_part[i];
    if (u) atomicAdd(out, u);
  }
}

__global__ void k_scalars_init(PeelScalars *sc, int32_t n, const unsigned long long *sum_all) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->cnt[0] = (unsigned long long)n;
    sc->cnt[1] = 0;
    sc->nu = sc->nu_big = sc->deg_peel = sc->deg_keep = sc->nlt = sc->trims = sc->nitems = 0;
    sc->sum2 = *sum_all;                // the reduce of S_0 = V
    sc->tau_lo = sc->tau_hi = 0;
    sc->tau_den = 1;
    sc->f = sc->s = sc->best_f = 0;
    sc->best_i = -1;
    sc->best_s = 1;
    sc->round = 0;
    sc->phase = STEP_PEEL;
    sc->bound = n;
    sc->ncut = 0;
    sc->nonprefix = 0;
  }
}

__device__ __forceinline__ u128 tau_num(const PeelScalars *sc) {
  return ((u128)sc->tau_hi << 64) | (u128)sc->tau_lo;
}

// the survivors are exactly the ids below bound (distinct ids, as many as
// the bound): then a vertex is alive iff its id is below the bound
__device__ __forceinline__ bool prefix_alive(const PeelScalars *sc, int cb) {
  return sc->cnt[cb] == (unsigned long long)sc->bound;
}

// pull re-sums the survivors' rows; with prefix survivors that is one
// binary search per survivor, otherwise a pass over their rows
__device__ __forceinline__ bool pull_step(const PeelScalars *sc, int cb) {
  if (prefix_alive(sc, cb)) return sc->deg_peel > sc->cnt[cb];
  return sc->deg_peel * PUSH_COST > sc->deg_keep;
}

// one bit per vertex, set while it is alive (n/8 bytes: stays in L2)
__device__ __forceinline__ bool is_alive(const uint32_t *__restrict__ alive, int32_t x) {
  return (alive[x >> 5] >> (x & 31)) & 1u;
}

// clear the alive bits of the lanes that remove their vertex. Every lane of
// the wavefront calls this (v < 0: no vertex); lanes with vertices of one
// 32-bit word next to each other merge their bits first, so a run of
// consecutive vertices costs one atomic per word.
__device__ __forceinline__ void clear_alive(uint32_t *alive, int32_t v, bool out) {
  const int lane = threadIdx.x & 63;
  const int32_t word = v >= 0 ? (v >> 5) : -1 - lane;
  uint32_t bits = out ? 1u << (v & 31) : 0u;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t w2 = __shfl_down(word, off);
    const uint32_t b2 = __shfl_down(bits, off);
    if (lane + off < 64 && w2 == word) bits |= b2;
  }
  const int32_t prev = __shfl_up(word, 1);
  if (bits && (lane == 0 || prev != word)) atomicAnd(&alive[word], ~bits);
}

// LPO: the survivors lighter than g(S) (w_u |S| < f(S)), one atomic per block
__global__ __launch_bounds__(BLOCK) void k_count_lt(const int32_t *__restrict__ la, int ca, PeelScalars *sc,
                                                    const int64_t *__restrict__ w) {
  __shared__ unsigned long long s_n;
  if (sc->round == 0) return;          // no trimming before the first peeling step
  const unsigned long long count = sc->cnt[ca];
  const u128 f = (u128)(uint64_t)sc->f, sz = (u128)(uint64_t)sc->s;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  unsigned long long c = 0;
  for (unsigned long long i = (unsigned long long)blockIdx.x * BLOCK + threadIdx.x; i < count;
       i += (unsigned long long)gridDim.x * BLOCK)
    if ((u128)(uint64_t)w[la[i]] * sz < f) c++;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(&s_n, c);
  __syncthreads();
  if (threadIdx.x == 0 && s_n) atomicAdd(&sc->nlt, s_n);
}

// one thread: the kind of the next step. A trimming step while (LPO) some
// survivor of the round is lighter than g(S); otherwise the round is over:
// its set is a candidate for the densest, and the next round starts with
// tau_max refined (GPO, LPO) from g of that set.
__device__ void next_phase(PeelScalars *sc, int32_t mode, int32_t k, int32_t num, int32_t den) {
  const long long f = sc->f, s = sc->s;
  if (s == 0) { sc->phase = STEP_DONE; return; }
  if (mode == MODE_LPO && sc->round > 0 && sc->nlt > 0) {
    sc->phase = STEP_TRIM;
    sc->trims++;
    sc->nlt = 0;
    return;
  }
  sc->nlt = 0;
  if (sc->best_i < 0 || (u128)(uint64_t)f * (u128)(uint64_t)sc->best_s >
                            (u128)(uint64_t)sc->best_f * (u128)(uint64_t)s) {
    sc->best_i = sc->round;
    sc->best_f = f;
    sc->best_s = s;
  }
  if (mode != MODE_PLAIN) {            // tau_max = max(tau_max, g / (k (1 + eps)))
    const u128 nA = (u128)(uint64_t)f * (u128)(uint64_t)den;
    const u128 nB = (u128)(uint64_t)s * (u128)(uint64_t)k * (u128)(uint64_t)(den + num);
    if (nA * (u128)sc->tau_den > tau_num(sc) * nB) {
      sc->tau_lo = (unsigned long long)nA;
      sc->tau_hi = (unsigned long long)(nA >> 64);
      sc->tau_den = (unsigned long long)nB;
    }
  }
  sc->round++;
  sc->phase = STEP_PEEL;
}

__global__ void k_phase(PeelScalars *sc, int32_t mode, int32_t k, int32_t num, int32_t den) {
  if (threadIdx.x == 0 && blockIdx.x == 0) next_phase(sc, mode, k, num, den);
}

// exclusive prefix sum over the block of one value per thread
__device__ __forceinline__ unsigned block_excl_scan(unsigned x, unsigned *s_w, unsigned *total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned v = x;
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned y = __shfl_up(v, off);
    if (lane >= off) v += y;
  }
  if (lane == 63) s_w[wid] = v;
  __syncthreads();
  unsigned before = 0, all = 0;
  for (int i = 0; i < BLOCK / 64; i++) {
    if (i < wid) before += s_w[i];
    all += s_w[i];
  }
  __syncthreads();
  *total = all;
  return before + v - x;
}

// decide: a block takes CHUNK alive vertices at a time (PER per thread,
// strided so loads coalesce), tests each, and appends the peeled and the
// surviving ones with one reservation per list and chunk; the degree sums
// of both sets choose how the weights are updated. A removed vertex gets
// its round and loses its alive bit.
constexpr int PER = 8, CHUNK = PER * BLOCK;

__global__ __launch_bounds__(BLOCK) void k_decide(const int32_t *__restrict__ la, int ca,
                                                  int32_t *__restrict__ lb, int cb, int32_t *__restrict__ ul,
                                                  int32_t n_total, PeelScalars *sc, const int64_t *__restrict__ w,
                                                  const int64_t *__restrict__ ptr, int32_t *__restrict__ rnd_in,
                                                  uint32_t *__restrict__ alive,
                                                  int32_t k, int32_t num, int32_t den) {
  __shared__ unsigned s_w[BLOCK / 64];
  __shared__ unsigned long long s_base[3];
  __shared__ unsigned long long s_deg[2][BLOCK / 64];
  __shared__ int s_top[BLOCK / 64];
  const int phase = sc->phase;
  if (phase == STEP_DONE) return;
  const int32_t round = sc->round;
  const unsigned long long count = sc->cnt[ca];
  // peeling: w <= max(tau_max, k (1 + eps) g), i.e. w tau_den <= tau or
  // w |S| den <= k (den + num) f; trimming: w < max(tau_max, g), i.e.
  // w tau_den < tau or w |S| < f
  const bool trim = phase == STEP_TRIM;
  const u128 rhs = trim ? (u128)(uint64_t)sc->f : (u128)(uint64_t)k * (u128)(uint64_t)(den + num) * (u128)(uint64_t)sc->f;
  const u128 scale = trim ? (u128)(uint64_t)sc->s : (u128)(uint64_t)sc->s * (u128)(uint64_t)den;
  const u128 tau = tau_num(sc), tden = (u128)sc->tau_den;
  int32_t top = 0;                  // 1 + the largest surviving id seen by this thread
  unsigned long long dp = 0, dk = 0;   // incidences of its removed and surviving vertices
  for (unsigned long long c0 = (unsigned long long)blockIdx.x * CHUNK; c0 < count;
       c0 += (unsigned long long)gridDim.x * CHUNK) {
    int32_t v[PER];
    unsigned peel_bits = 0, big_bits = 0, np = 0, nb = 0, nk = 0;
#pragma unroll
    for (int j = 0; j < PER; j++) {
      const unsigned long long idx = c0 + (unsigned long long)j * BLOCK + threadIdx.x;
      v[j] = idx < count ? (la ? la[idx] : (int32_t)idx) : -1;   // no list: the identity (first step)
    }
#pragma unroll
    for (int j = 0; j < PER; j++) {
      if (v[j] < 0) continue;
      const unsigned long long d = (unsigned long long)(ptr[v[j] + 1] - ptr[v[j]]);
      const u128 wv = (u128)(uint64_t)w[v[j]];
      const bool out = trim ? (wv * tden < tau || wv * scale < rhs) : (wv * tden <= tau || wv * scale <= rhs);
      if (out) {
        peel_bits |= 1u << j;
        if (d > SMALL_PUSH) { big_bits |= 1u << j; nb++; } else np++;
        dp += d;
      } else {
        nk++;
        dk += d;
      }
    }
    unsigned tp, tb, tk;
    const unsigned op = block_excl_scan(np, s_w, &tp);
    const unsigned ob = block_excl_scan(nb, s_w, &tb);
    const unsigned ok = block_excl_scan(nk, s_w, &tk);
    if (threadIdx.x == 0) {
      s_base[0] = tp ? atomicAdd(&sc->nu, (unsigned long long)tp) : 0ull;
      s_base[1] = tk ? atomicAdd(&sc->cnt[cb], (unsigned long long)tk) : 0ull;
      s_base[2] = tb ? atomicAdd(&sc->nu_big, (unsigned long long)tb) : 0ull;
    }
    __syncthreads();
    unsigned long long pu = s_base[0] + op, pk = s_base[1] + ok, pb = s_base[2] + ob;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; j++) {
      clear_alive(alive, v[j], (peel_bits >> j) & 1u);
      if (v[j] < 0) continue;
      if ((peel_bits >> j) & 1u) {
        rnd_in[v[j]] = round;
        if ((big_bits >> j) & 1u) ul[n_total - 1 - pb++] = v[j];   // large rows fill the list from its end
        else ul[pu++] = v[j];
      } else {
        lb[pk++] = v[j];
        top = max(top, v[j] + 1);
      }
    }
  }
  // the block's degree totals and largest survivor, one atomic each
  for (int off = 32; off > 0; off >>= 1) {
    dp += __shfl_xor(dp, off);
    dk += __shfl_xor(dk, off);
    top = max(top, __shfl_xor(top, off));
  }
  if ((threadIdx.x & 63) == 0) {
    s_deg[0][threadIdx.x >> 6] = dp;
    s_deg[1][threadIdx.x >> 6] = dk;
    s_top[threadIdx.x >> 6] = top;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, b = 0;
    int t = 0;
    for (int i = 0; i < BLOCK / 64; i++) {
      a += s_deg[0][i];
      b += s_deg[1][i];
      t = max(t, s_top[i]);
    }
    if (a) atomicAdd(&sc->deg_peel, a);
    if (b) atomicAdd(&sc->deg_keep, b);
    if (t) atomicMax(&sc->bound, t);
  }
}

// the pull's work list when the survivors are not the ids below the bound:
// every survivor's row in pieces of PIECE incidences (a row of many pieces
// is listed by the whole wavefront); reserved once per block and chunk
constexpr int IPER = 4, ICHUNK = IPER * BLOCK;
__device__ __forceinline__ void list_items(const int32_t *__restrict__ lb, int cb, PeelScalars *sc,
                                           const int64_t *__restrict__ ptr, unsigned long long *__restrict__ items) {
  __shared__ unsigned s_w[BLOCK / 64];
  __shared__ unsigned long long s_base;
  const unsigned long long count = sc->cnt[cb];
  for (unsigned long long c0 = (unsigned long long)blockIdx.x * ICHUNK; c0 < count;
       c0 += (unsigned long long)gridDim.x * ICHUNK) {
    int32_t v[IPER];
    uint32_t pcs[IPER];
    unsigned ni = 0;
#pragma unroll
    for (int j = 0; j < IPER; j++) {
      const unsigned long long idx = c0 + (unsigned long long)j * BLOCK + threadIdx.x;
      v[j] = idx < count ? lb[idx] : -1;
      pcs[j] = v[j] < 0 ? 0u : (uint32_t)((ptr[v[j] + 1] - ptr[v[j]] + PIECE - 1) / PIECE);
      ni += pcs[j];
    }
    unsigned ti;
    const unsigned oi = block_excl_scan(ni, s_w, &ti);
    if (threadIdx.x == 0) s_base = ti ? atomicAdd(&sc->nitems, (unsigned long long)ti) : 0ull;
    __syncthreads();
    unsigned long long pi = s_base + oi;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPER; j++) {
      const bool many = pcs[j] > FEW_PIECES;
      unsigned long long first = pi;
      if (many) pi += pcs[j];
      else
        for (uint32_t q = 0; q < pcs[j]; q++) items[pi++] = ((unsigned long long)v[j] << 32) | q;
      for (unsigned long long ball = __ballot(many); ball; ball &= ball - 1) {
        const int l = __ffsll((unsigned long long)ball) - 1;
        const unsigned long long row = (unsigned long long)(uint32_t)__shfl(v[j], l) << 32;
        const unsigned long long at = __shfl(first, l);
        const uint32_t cnt = __shfl(pcs[j], l);
        for (uint32_t q = threadIdx.x & 63; q < cnt; q += 64) items[at + q] = row | q;
      }
    }
  }
}

// push: the removed vertices subtract their edge weights from the
// neighbours still alive; a thread per vertex with a small row, a
// wavefront per vertex with a large one. Runs while the removed vertices
// have few incidences next to the survivors' (pull_step).
__device__ __forceinline__ void push_updates(const int32_t *__restrict__ ul, int32_t n_total, PeelScalars *sc, int cb,
                                             const int64_t *__restrict__ ptr, const int32_t *__restrict__ nbr,
                                             const int64_t *__restrict__ wt, const uint32_t *__restrict__ alive,
                                             int64_t *__restrict__ w) {
  const unsigned long long nu = sc->nu, nb = sc->nu_big;
  const int32_t bound = sc->bound;
  const bool prefix = prefix_alive(sc, cb);
  for (unsigned long long i = (unsigned long long)blockIdx.x * BLOCK + threadIdx.x; i < nu;
       i += (unsigned long long)gridDim.x * BLOCK) {
    const int32_t u = ul[i];
    for (int64_t j = ptr[u]; j < ptr[u + 1]; j++) {
      const int32_t x = nbr[j];
      if (x < bound && (prefix || is_alive(alive, x)))
        atomicAdd((unsigned long long *)&w[x], (unsigned long long)(-(wt ? wt[j] : 1ll)));
    }
  }
  const int lane = threadIdx.x & 63;
  for (unsigned long long i = ((unsigned long long)blockIdx.x * BLOCK + threadIdx.x) >> 6; i < nb;
       i += ((unsigned long long)gridDim.x * BLOCK) >> 6) {
    const int32_t u = ul[n_total - 1 - i];
    const int64_t b = ptr[u], e = ptr[u + 1];
    for (int64_t j = b + lane; j < e; j += 64) {
      const int32_t x = nbr[j];
      if (x < bound && (prefix || is_alive(alive, x)))
        atomicAdd((unsigned long long *)&w[x], (unsigned long long)(-(wt ? wt[j] : 1ll)));
    }
  }
}

// pull: the survivors' weights restart from a. When the survivors are the
// ids below the bound (as the renumbering makes them after the first round),
// a survivor's alive neighbours are the head of its sorted row: a binary
// search finds its end, and the weight is its length (DG) or a difference
// of the running weight sums. Otherwise each piece of PIECE incidences of a
// survivor's row (listed by decide) is summed over the alive neighbours by
// one wavefront and added with one atomic, so hub rows spread over many
// wavefronts.
__device__ __forceinline__ void pull_reset(const int32_t *__restrict__ lb, int cb, PeelScalars *sc,
                                           const int64_t *__restrict__ a, const int64_t *__restrict__ ptr,
                                           const int32_t *__restrict__ nbr, const int64_t *__restrict__ wcum,
                                           int64_t *__restrict__ w) {
  const unsigned long long count = sc->cnt[cb];
  const bool prefix = prefix_alive(sc, cb);
  const int32_t bound = sc->bound;
  for (unsigned long long i = (unsigned long long)blockIdx.x * BLOCK + threadIdx.x; i < count;
       i += (unsigned long long)gridDim.x * BLOCK) {
    const int32_t v = lb[i];
    int64_t x = a ? a[v] : 0;
    if (prefix) {
      // rows are sorted: the alive neighbours are the entries below the bound
      const int64_t b = ptr[v];
      int64_t lo = b, hi = ptr[v + 1];
      while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (nbr[mid] < bound) lo = mid + 1;
        else hi = mid;
      }
      if (!wcum) x += lo - b;
      else if (lo > b) x += wcum[lo - 1] - (b > 0 ? wcum[b - 1] : 0);
    }
    w[v] = x;
  }
}

// the first launch of the update: push, or the pull's reset (and its work
// list when the survivors are not the ids below the bound); the role is the
// same for the whole grid
__global__ __launch_bounds__(BLOCK) void k_update(const int32_t *__restrict__ ul, int32_t n_total,
                                                  const int32_t *__restrict__ lb, int cb, PeelScalars *sc,
                                                  const int64_t *__restrict__ a, const int64_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ nbr, const int64_t *__restrict__ wt,
                                                  const int64_t *__restrict__ wcum, const uint32_t *__restrict__ alive,
                                                  unsigned long long *__restrict__ items, int64_t *__restrict__ w) {
  if (!pull_step(sc, cb)) {
    push_updates(ul, n_total, sc, cb, ptr, nbr, wt, alive, w);
    return;
  }
  if (!prefix_alive(sc, cb)) list_items(lb, cb, sc, ptr, items);
  pull_reset(lb, cb, sc, a, ptr, nbr, wcum, w);
}

__global__ __launch_bounds__(BLOCK) void k_update_pull(const unsigned long long *__restrict__ items, PeelScalars *sc,
                                                       int cb,
                                                       const int64_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ nbr,
                                                       const int64_t *__restrict__ wt,
                                                       const uint32_t *__restrict__ alive, int64_t *__restrict__ w) {
  if (!pull_step(sc, cb) || prefix_alive(sc, cb)) return;   // prefix survivors: done by the reset
  const unsigned long long count = sc->nitems;
  const int32_t bound = sc->bound;
  const int lane = threadIdx.x & 63;
  const unsigned long long waves = ((unsigned long long)gridDim.x * BLOCK) >> 6;
  for (unsigned long long it = ((unsigned long long)blockIdx.x * BLOCK + threadIdx.x) >> 6; it < count; it += waves) {
    const unsigned long long item = items[it];
    const int32_t v = (int32_t)(item >> 32);
    const int64_t b = ptr[v] + (int64_t)(item & 0xffffffffull) * PIECE;
    const int64_t e = min(ptr[v + 1], b + PIECE);
    if (nbr[b] >= bound) continue;   // rows are sorted: every neighbour in the piece is gone
    unsigned long long s = 0;
    int32_t xs[PIECE / 64];
#pragma unroll
    for (int t = 0; t < PIECE / 64; t++) {
      const int64_t j = b + lane + 64 * t;
      xs[t] = j < e ? nbr[j] : bound;
    }
#pragma unroll
    for (int t = 0; t < PIECE / 64; t++)
      if (xs[t] < bound && is_alive(alive, xs[t])) s += (unsigned long long)(wt ? wt[b + lane + 64 * t] : 1ll);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0 && s) atomicAdd((unsigned long long *)&w[v], s);
  }
}

__global__ __launch_bounds__(BLOCK) void k_reduce(const int32_t *__restrict__ list, int cl, PeelScalars *sc,
                                                  const int64_t *__restrict__ a, const int64_t *__restrict__ w) {
  __shared__ unsigned long long s_part[BLOCK / 64];
  const unsigned long long count = sc->cnt[cl];
  unsigned long long s = 0;
  for (unsigned long long i = (unsigned long long)blockIdx.x * BLOCK + threadIdx.x; i < count;
       i += (unsigned long long)gridDim.x * BLOCK) {
    const int32_t v = list[i];
    s += (unsigned long long)w[v] + (a ? (unsigned long long)a[v] : 0ull);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int i = 0; i < BLOCK / 64; i++) t += s_part[i];
    if (t) atomicAdd(&sc->sum2, t);
  }
}

// close a step: survivors are in list cl; the next step fills 1 - cl. The
// record of the round is rewritten by every step of it (the last, after
// trimming, stays).
__global__ void k_end(int cl, PeelScalars *sc, int64_t *sizes, int64_t *fs, int32_t cap, int32_t mode, int32_t k,
                      int32_t num, int32_t den) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (sc->phase == STEP_DONE) return;
  const int32_t round = sc->round;
  const long long f = (long long)(sc->sum2 / 2ull), s = (long long)sc->cnt[cl];
  if (round < cap) { sizes[round] = s; fs[round] = f; }
  // the step removed the ids in [bound, the previous bound) when its
  // survivors are the ids below the bound
  if ((unsigned long long)sc->bound != sc->cnt[cl]) sc->nonprefix = 1;
  if (sc->ncut < MAX_CUTS) {
    sc->cut[sc->ncut] = sc->bound;
    sc->cut_round[sc->ncut] = round;
  }
  sc->ncut++;
  sc->f = f;
  sc->s = s;
  sc->sum2 = 0;
  sc->nu = sc->nu_big = 0;
  sc->deg_peel = sc->deg_keep = 0;
  sc->nitems = 0;
  sc->bound = 0;
  sc->cnt[1 - cl] = 0;
  // without trimming the next step's kind needs nothing more: pick it here
  // (with trimming, the count of light survivors comes first)
  if (mode != MODE_LPO) next_phase(sc, mode, k, num, den);
}

// end of a run: the peel rounds in the caller's ids, with coalesced
// stores. When every step left the ids below its bound, a vertex's round
// follows from its internal id and the steps' bounds (the first step whose
// bound it is not below); otherwise a gather through the id map.
__global__ __launch_bounds__(BLOCK) void k_export(int32_t n, const int32_t *__restrict__ inv,
                                                  const int32_t *__restrict__ rnd_in, const PeelScalars *sc,
                                                  int32_t *__restrict__ rnd) {
  __shared__ int s_cut[MAX_CUTS], s_round[MAX_CUTS];
  const int ncut = sc->ncut;
  const bool by_cuts = !sc->nonprefix && ncut <= MAX_CUTS;
  if (by_cuts) {
    for (int i = threadIdx.x; i < ncut; i += BLOCK) {
      s_cut[i] = sc->cut[i];
      s_round[i] = sc->cut_round[i];
    }
    __syncthreads();
  }
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
    const int32_t x = inv[v];
    if (by_cuts) {
      int lo = 0, hi = ncut - 1;   // the last step's bound is 0: some step's bound is not above x
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x >= s_cut[mid]) hi = mid;
        else lo = mid + 1;
      }
      rnd[v] = s_round[lo];
    } else {
      rnd[v] = rnd_in[x];
    }
  }
}

unsigned grid_for(int64_t items, int64_t per_block, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + per_block - 1) / per_block, cap));
}

}  // namespace
}  // namespace kws

struct kws_dsd_graph {
  int32_t n = 0;
  int64_t m = 0;
  int metric = 0;
  int64_t *ptr = nullptr;          // [n + 1] incidence offsets
  int32_t *nbr = nullptr;          // [2m]
  int64_t *wt = nullptr;           // [2m] edge weights (none for DG)
  int64_t *wcum = nullptr;         // [2m] running sum of wt over all rows (none for DG)
  int64_t *a = nullptr;            // [n] vertex weights (FD only)
  int32_t *big = nullptr;          // vertices whose row is summed by a wavefront
  int32_t nbig = 0;
  int64_t *w0 = nullptr;           // [n] peeling weights in G (start of every run)
  unsigned long long *sum_all = nullptr;   // 2 f(V)
  int64_t *w = nullptr;            // [n] peeling weights
  int32_t *rnd = nullptr;          // [n] round of removal, in the caller's ids
  int32_t *rnd_in = nullptr;       // [n] round of removal, in internal ids
  int32_t *inv = nullptr;          // [n] internal id of each caller's id
  int32_t *list[2] = {nullptr, nullptr};
  int32_t *ul = nullptr;           // [n] peeled in the current round
  uint32_t *alive = nullptr;       // [(n + 31) / 32] alive bits
  unsigned long long *items = nullptr;   // [n + 2m / PIECE] pull items: vertex << 32 | piece
  kws::PeelScalars *sc = nullptr;
  int64_t *d_sizes = nullptr, *d_f = nullptr;
  int32_t d_cap = 0;
  bool has_run = false;            // rnd holds the rounds of a finished run
  hipStream_t stream = nullptr;
};

namespace {

void dsd_release(kws_dsd_graph *g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  void *ps[] = {g->ptr, g->nbr, g->wt, g->wcum, g->a, g->big, g->w0, g->w, g->rnd, g->rnd_in, g->inv, g->list[0], g->list[1], g->ul, g->alive, g->items, g->sum_all, g->sc,
                g->d_sizes, g->d_f};
  for (void *p : ps) kws::dev_free(p);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

template <class T>
kws_status dev_array(T **p, size_t count, const char *what) {
  *p = (T *)kws::dev_alloc(sizeof(T) * std::max<size_t>(count, 1));
  if (!*p) return kws::fail(KWS_ENOMEM, "device allocation for %s (%zu bytes)", what, sizeof(T) * count);
  return KWS_OK;
}

// event timing of one kernel class
// event pairs of the timed kernel classes of one run, read after its last
// synchronisation (no wait while steps are enqueued)
enum { DSD_DECIDE = 0, DSD_UPDATE = 1, DSD_REDUCE = 2 };
struct DsdEvents {
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  ~DsdEvents() {
    for (Rec &r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  }
  void collect(kws_dsd_summary &sum) {
    double *ms[3] = {&sum.decide_ms, &sum.update_ms, &sum.reduce_ms};
    int64_t *n[3] = {&sum.decide_launches, &sum.update_launches, &sum.reduce_launches};
    for (Rec &r : recs) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) { *ms[r.cls] += t; (*n[r.cls])++; }
    }
  }
};

struct DsdTimer {
  DsdEvents *log;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  DsdTimer(bool on, int cls_, hipStream_t s_, DsdEvents *log_) : log(nullptr), cls(cls_), s(s_) {
    if (on && hipEventCreate(&a) == hipSuccess) {
      log = log_;
      (void)hipEventRecord(a, s);   // a failed record makes this pair's elapsed time fail: it is skipped
    }
  }
  ~DsdTimer() {
    if (!log) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
    (void)hipEventRecord(b, s);
    log->recs.push_back({cls, a, b});
  }
};

}  // namespace

extern "C" {

kws_status kws_dsd_load(const kws_dsd_desc *d, kws_dsd_graph **out) {
  using namespace kws;
  clear_error();
  if (!d || !out) return fail(KWS_EINVAL, "null argument");
  *out = nullptr;
  if (d->n < 0 || d->m < 0 || (d->m > 0 && (!d->src || !d->dst))) return fail(KWS_EINVAL, "bad graph size or arrays");
  if (d->metric < KWS_DSD_DG || d->metric > KWS_DSD_FD) return fail(KWS_EINVAL, "unknown metric %d", d->metric);
  if (d->metric == KWS_DSD_DW && d->m > 0 && !d->edge_w) return fail(KWS_EINVAL, "DW needs edge weights");
  if (d->metric == KWS_DSD_FD && d->n > 0 && !d->vertex_w) return fail(KWS_EINVAL, "FD needs vertex weights");
  const int32_t n = d->n;
  const int64_t m = d->m;
  std::vector<int32_t> deg((size_t)n, 0);
  u128 tot_e = 0, tot_v = 0;
  for (int64_t e = 0; e < m; e++) {
    const int32_t u = d->src[e], v = d->dst[e];
    if (u < 0 || u >= n || v < 0 || v >= n) return fail(KWS_EINVAL, "edge %lld has an endpoint out of range", (long long)e);
    if (u == v) return fail(KWS_EINVAL, "edge %lld is a self-loop", (long long)e);
    if (d->metric == KWS_DSD_DW) {
      if (d->edge_w[e] < 0) return fail(KWS_EINVAL, "negative edge weight at %lld", (long long)e);
      tot_e += (u128)(uint64_t)d->edge_w[e];
    }
    deg[u]++;
    deg[v]++;
  }
  if (d->metric == KWS_DSD_FD)
    for (int32_t v = 0; v < n; v++) {
      if (d->vertex_w[v] < 0) return fail(KWS_EINVAL, "negative vertex weight at %d", v);
      tot_v += (u128)(uint64_t)d->vertex_w[v];
    }
  if (tot_e >= ((u128)1 << 55) || tot_v >= ((u128)1 << 55)) return fail(KWS_EOVERFLOW, "weights sum to 2^55 or more");
  // FD edge weight by source degree: 1 / ln(deg + 5) in 2^-24 units
  int32_t maxdeg = 0;
  for (int32_t v = 0; v < n; v++) maxdeg = std::max(maxdeg, deg[v]);
  std::vector<int64_t> fd_table;
  if (d->metric == KWS_DSD_FD) {
    fd_table.resize((size_t)maxdeg + 1);
    for (int32_t x = 0; x <= maxdeg; x++) fd_table[x] = std::llround(16777216.0 / std::log((double)x + 5.0));
  }
  // Internal ids by descending initial peeling weight w_u(V) (ties by id):
  // the first round keeps exactly the heaviest vertices, so its survivors
  // are the smallest ids, and the later rounds' survivors, the dense part,
  // stay among them; their alive bits and weights sit together and a
  // sorted row holds them at its start.
  std::vector<int32_t> perm((size_t)n), inv((size_t)n);
  {
    std::vector<uint64_t> w0((size_t)n);
    for (int32_t v = 0; v < n; v++) w0[(size_t)v] = (uint64_t)deg[(size_t)v];
    if (d->metric != KWS_DSD_DG) {
      std::fill(w0.begin(), w0.end(), 0ull);
      for (int64_t e = 0; e < m; e++) {
        const int32_t u = d->src[e], v = d->dst[e];
        const uint64_t c = d->metric == KWS_DSD_DW ? (uint64_t)d->edge_w[e] : (uint64_t)fd_table[(size_t)deg[(size_t)u]];
        w0[(size_t)u] += c;
        w0[(size_t)v] += c;
      }
      if (d->metric == KWS_DSD_FD)
        for (int32_t v = 0; v < n; v++) w0[(size_t)v] += (uint64_t)d->vertex_w[v];
    }
    // stable LSD radix sort of the ids by ~w0 (descending w0, ties by id)
    uint64_t top = 0;
    for (int32_t v = 0; v < n; v++) top = std::max(top, w0[(size_t)v]);
    std::vector<int32_t> tmp((size_t)n);
    for (int32_t v = 0; v < n; v++) perm[(size_t)v] = v;
    for (int shift = 0; shift < 64 && (top >> shift) != 0; shift += 16) {
      std::vector<int64_t> at(65537, 0);
      for (int32_t i = 0; i < n; i++) at[(((top - w0[(size_t)perm[(size_t)i]]) >> shift) & 0xffff) + 1]++;
      for (size_t b = 1; b < at.size(); b++) at[b] += at[b - 1];
      for (int32_t i = 0; i < n; i++) {
        const int32_t v = perm[(size_t)i];
        tmp[(size_t)at[((top - w0[(size_t)v]) >> shift) & 0xffff]++] = v;
      }
      perm.swap(tmp);
    }
    for (int32_t i = 0; i < n; i++) inv[(size_t)perm[(size_t)i]] = i;
  }
  std::vector<int32_t> ideg((size_t)n);
  std::vector<int64_t> ptr((size_t)n + 1, 0);
  std::vector<int32_t> big;
  for (int32_t i = 0; i < n; i++) {
    ideg[(size_t)i] = deg[(size_t)perm[(size_t)i]];
    ptr[i + 1] = ptr[i] + ideg[(size_t)i];
    if (ideg[(size_t)i] > SMALL_DEG) big.push_back(i);
  }
  std::vector<int64_t> ia;
  if (d->metric == KWS_DSD_FD) {
    ia.resize((size_t)n);
    for (int32_t i = 0; i < n; i++) ia[(size_t)i] = d->vertex_w[perm[(size_t)i]];
  }

  kws_dsd_graph *g = new kws_dsd_graph();
  g->n = n;
  g->m = m;
  g->metric = d->metric;
  auto bail = [&](kws_status st) { dsd_release(g); return st; };
  if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(KWS_EDEVICE, "stream creation failed"));
  hipStream_t s = g->stream;
  kws_status st = KWS_OK;
  int32_t *d_src = nullptr, *d_dst = nullptr, *d_deg = nullptr;
  int64_t *d_ew = nullptr, *d_fd = nullptr, *d_vals = nullptr;
  unsigned long long *d_keys = nullptr, *d_sorted = nullptr;
  void *d_tmp = nullptr;
  auto cleanup = [&]() {
    dev_free(d_src); dev_free(d_dst); dev_free(d_deg); dev_free(d_ew); dev_free(d_fd);
    dev_free(d_vals); dev_free(d_keys); dev_free(d_sorted); dev_free(d_tmp);
  };
#define DSD_STEP(x) do { st = (x); if (st != KWS_OK) { cleanup(); return bail(st); } } while (0)
#define DSD_HIP(x) DSD_STEP((x) == hipSuccess ? KWS_OK : fail(KWS_EDEVICE, "%s failed", #x))
  DSD_STEP(dev_array(&g->ptr, (size_t)n + 1, "incidence offsets"));
  DSD_STEP(dev_array(&g->nbr, (size_t)(2 * m), "incidences"));
  if (d->metric != KWS_DSD_DG) DSD_STEP(dev_array(&g->wt, (size_t)(2 * m), "incidence weights"));
  if (d->metric == KWS_DSD_FD) DSD_STEP(dev_array(&g->a, (size_t)n, "vertex weights"));
  DSD_STEP(dev_array(&g->big, big.size(), "large rows"));
  DSD_STEP(dev_array(&g->w0, (size_t)n, "initial peeling weights"));
  DSD_STEP(dev_array(&g->w, (size_t)n, "peeling weights"));
  DSD_STEP(dev_array(&g->rnd, (size_t)n, "peel rounds"));
  DSD_STEP(dev_array(&g->rnd_in, (size_t)n, "peel rounds (internal ids)"));
  DSD_STEP(dev_array(&g->inv, (size_t)n, "id map"));
  DSD_STEP(dev_array(&g->list[0], (size_t)n, "alive list"));
  DSD_STEP(dev_array(&g->list[1], (size_t)n, "alive list"));
  DSD_STEP(dev_array(&g->ul, (size_t)n, "peeled list"));
  DSD_STEP(dev_array(&g->alive, ((size_t)n + 31) / 32, "alive bits"));
  DSD_STEP(dev_array(&g->items, (size_t)n + (size_t)(2 * m) / PIECE + 1, "pull items"));
  DSD_STEP(dev_array(&g->sc, 1, "peeling scalars"));
  DSD_STEP(dev_array(&g->sum_all, 1, "2 f(V)"));
  g->nbig = (int32_t)big.size();
  DSD_HIP(hipMemcpyAsync(g->ptr, ptr.data(), sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s));
  if (n > 0) DSD_HIP(hipMemcpyAsync(g->inv, inv.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
  if (!big.empty()) DSD_HIP(hipMemcpyAsync(g->big, big.data(), sizeof(int32_t) * big.size(), hipMemcpyHostToDevice, s));
  if (g->a) DSD_HIP(hipMemcpyAsync(g->a, ia.data(), sizeof(int64_t) * (size_t)n, hipMemcpyHostToDevice, s));
  if (m > 0) {
    const size_t inc = (size_t)(2 * m);
    DSD_STEP(dev_array(&d_src, (size_t)m, "edge sources"));
    DSD_STEP(dev_array(&d_dst, (size_t)m, "edge targets"));
    DSD_STEP(dev_array(&d_keys, inc, "incidence keys"));
    DSD_STEP(dev_array(&d_sorted, inc, "sorted incidence keys"));
    DSD_HIP(hipMemcpyAsync(d_src, d->src, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s));
    DSD_HIP(hipMemcpyAsync(d_dst, d->dst, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s));
    if (d->metric == KWS_DSD_DW) {
      DSD_STEP(dev_array(&d_ew, (size_t)m, "edge weights"));
      DSD_HIP(hipMemcpyAsync(d_ew, d->edge_w, sizeof(int64_t) * (size_t)m, hipMemcpyHostToDevice, s));
    }
    if (d->metric == KWS_DSD_FD) {
      DSD_STEP(dev_array(&d_fd, fd_table.size(), "FD weight table"));
      DSD_STEP(dev_array(&d_deg, (size_t)n, "degrees"));
      DSD_HIP(hipMemcpyAsync(d_fd, fd_table.data(), sizeof(int64_t) * fd_table.size(), hipMemcpyHostToDevice, s));
      DSD_HIP(hipMemcpyAsync(d_deg, ideg.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    }
    if (g->wt) DSD_STEP(dev_array(&d_vals, inc, "incidence weight keys"));
    k_keys<<<grid_for(m, BLOCK, 65536), BLOCK, 0, s>>>(d_src, d_dst, d_ew, m, d->metric, d_fd, d_deg, g->inv, d_keys,
                                                       d_vals);
    DSD_HIP(hipGetLastError());
    // sort by (row, neighbour): 32 bits of neighbour and the bits of a row id
    int end_bit = 32;
    while (end_bit < 64 && ((int64_t)1 << (end_bit - 32)) < (int64_t)n) end_bit++;
    size_t tmp_bytes = 0;
    if (g->wt) {
      DSD_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, d_keys, d_sorted, d_vals, g->wt, inc, 0, end_bit, s));
      DSD_STEP(dev_array((char **)&d_tmp, tmp_bytes, "sort scratch"));
      DSD_HIP(hipcub::DeviceRadixSort::SortPairs(d_tmp, tmp_bytes, d_keys, d_sorted, d_vals, g->wt, inc, 0, end_bit, s));
    } else {
      DSD_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_bytes, d_keys, d_sorted, inc, 0, end_bit, s));
      DSD_STEP(dev_array((char **)&d_tmp, tmp_bytes, "sort scratch"));
      DSD_HIP(hipcub::DeviceRadixSort::SortKeys(d_tmp, tmp_bytes, d_keys, d_sorted, inc, 0, end_bit, s));
    }
    k_unpack<<<grid_for((int64_t)inc, BLOCK, 65536), BLOCK, 0, s>>>(d_sorted, (int64_t)inc, g->nbr);
    DSD_HIP(hipGetLastError());
    if (g->wt) {
      // running sum of the weights in CSR order: a row prefix's weight is a
      // difference of two entries (totals stay below 2^55)
      DSD_STEP(dev_array(&g->wcum, inc, "incidence weight sums"));
      size_t scan_bytes = 0;
      DSD_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, g->wt, g->wcum, inc, s));
      if (scan_bytes > tmp_bytes) {
        DSD_HIP(hipStreamSynchronize(s));
        dev_free(d_tmp);
        d_tmp = nullptr;
        DSD_STEP(dev_array((char **)&d_tmp, scan_bytes, "scan scratch"));
      }
      DSD_HIP(hipcub::DeviceScan::InclusiveSum(d_tmp, scan_bytes, g->wt, g->wcum, inc, s));
    }
  }
  k_w0_small<<<grid_for(n, BLOCK, 65536), BLOCK, 0, s>>>(n, g->ptr, g->wt, g->a, g->w0);
  if (g->nbig && g->wt)
    k_w0_big<<<grid_for((int64_t)g->nbig * 64, BLOCK, 65536), BLOCK, 0, s>>>(g->big, g->nbig, g->ptr, g->wt, g->w0);
  DSD_HIP(hipMemsetAsync(g->sum_all, 0, sizeof(unsigned long long), s));
  k_sum_all<<<grid_for(n, BLOCK, 2048), BLOCK, 0, s>>>(n, g->a, g->w0, g->sum_all);
  DSD_HIP(hipGetLastError());
  DSD_HIP(hipStreamSynchronize(s));
  cleanup();
#undef DSD_HIP
#undef DSD_STEP
  *out = g;
  return KWS_OK;
}

void kws_dsd_free(kws_dsd_graph *g) { dsd_release(g); }

kws_status kws_dsd_peel(kws_dsd_graph *g, const kws_dsd_params *p, int32_t *peel_round, int64_t *sizes,
                        int64_t *f, int32_t cap, kws_dsd_summary *summary) {
  using namespace kws;
  clear_error();
  if (!g || !p) return fail(KWS_EINVAL, "null argument");
  if (p->k < 1 || p->k > 64 || p->eps_num < 0 || p->eps_num > 1000 || p->eps_den < 1 || p->eps_den > 1000)
    return fail(KWS_EINVAL, "k must be 1..64, eps_num 0..1000, eps_den 1..1000");
  // every step must peel a vertex: the mean peeling weight is at most 2 g
  // (each edge weighs on both endpoints), so k (1 + eps) >= 2 guarantees it
  if ((int64_t)p->k * (p->eps_den + p->eps_num) < 2 * (int64_t)p->eps_den)
    return fail(KWS_EINVAL, "k (1 + eps) = %d (1 + %d/%d) is below 2: a peeling round may remove nothing", p->k,
                p->eps_num, p->eps_den);
  if (p->mode < KWS_DSD_PLAIN || p->mode > KWS_DSD_LPO) return fail(KWS_EINVAL, "unknown peeling mode %d", p->mode);
  if (p->profile_classes < 0 || p->profile_classes > 7) return fail(KWS_EINVAL, "profile_classes must be 0..7");
  if ((sizes || f) && cap < 1) return fail(KWS_EINVAL, "cap must be >= 1 with sizes or f");

  hipStream_t s = g->stream;
  const int32_t n = g->n;
  // device record of the rounds: enough for eps > 0 at any size; more is
  // reallocated when a run needs it
  const int32_t want_cap = std::max<int32_t>(4096, std::min<int32_t>(n + 2, std::max<int32_t>(cap, 0)));
  if (g->d_cap < want_cap) {
    dev_free(g->d_sizes);
    dev_free(g->d_f);
    g->d_sizes = g->d_f = nullptr;
    g->d_cap = 0;
    KWS_TRY(dev_array(&g->d_sizes, (size_t)want_cap, "round sizes"));
    KWS_TRY(dev_array(&g->d_f, (size_t)want_cap, "round f"));
    g->d_cap = want_cap;
  }
  kws_dsd_summary sum{};
  // profile 0: no events; otherwise events around the classes of
  // profile_classes (bit 0 decide, 1 update, 2 reduce; 0 = every class)
  const int pmask = p->profile ? (p->profile_classes ? p->profile_classes : 7) : 0;
  const bool t_dec = pmask & 1, t_upd = (pmask >> 1) & 1, t_red = (pmask >> 2) & 1;
  DsdEvents evlog;
  const int64_t resident = 2048;
  KWS_HIP(hipGetLastError());
  g->has_run = false;
  k_scalars_init<<<1, 64, 0, s>>>(g->sc, n, g->sum_all);
  k_start<<<grid_for(n, BLOCK, 65536), BLOCK, 0, s>>>(n, g->w0, g->w, g->rnd_in, g->alive);
  k_end<<<1, 64, 0, s>>>(0, g->sc, g->d_sizes, g->d_f, g->d_cap, p->mode, p->k, p->eps_num, p->eps_den);
  KWS_HIP(hipGetLastError());
  // Steps are enqueued without waiting: the device decides whether a step
  // peels (a new round), trims (LPO) or, once the set is empty, does
  // nothing. Every real step removes a vertex, so there are at most n.
  int64_t known = n;   // an upper bound of |S| (read back every few steps)
  int64_t step = 0;
  while (known > 0) {
    if (step > (int64_t)n + 1) return fail(KWS_EDEVICE, "peeling did not finish in %d steps", n + 1);
    step++;
    const int ca = (int)((step - 1) & 1), cb = (int)(step & 1);
    if (p->mode == KWS_DSD_LPO) {   // otherwise k_end has picked the step's kind
      k_count_lt<<<grid_for(known, BLOCK, resident), BLOCK, 0, s>>>(g->list[ca], ca, g->sc, g->w);
      k_phase<<<1, 64, 0, s>>>(g->sc, p->mode, p->k, p->eps_num, p->eps_den);
    }
    {
      DsdTimer t(t_dec, DSD_DECIDE, s, &evlog);
      k_decide<<<grid_for(known, CHUNK, resident), BLOCK, 0, s>>>(step == 1 ? nullptr : g->list[ca], ca, g->list[cb],
                                                                   cb, g->ul, n, g->sc,
                                                                   g->w, g->ptr, g->rnd_in, g->alive, p->k,
                                                                   p->eps_num, p->eps_den);
    }
    {
      DsdTimer t(t_upd, DSD_UPDATE, s, &evlog);
      k_update<<<grid_for(known * 64, BLOCK, resident), BLOCK, 0, s>>>(g->ul, n, g->list[cb], cb, g->sc, g->a, g->ptr,
                                                                       g->nbr, g->wt, g->wcum, g->alive, g->items, g->w);
      k_update_pull<<<(unsigned)resident, BLOCK, 0, s>>>(g->items, g->sc, cb, g->ptr, g->nbr, g->wt, g->alive, g->w);
    }
    {
      DsdTimer t(t_red, DSD_REDUCE, s, &evlog);
      k_reduce<<<grid_for(known, BLOCK, resident), BLOCK, 0, s>>>(g->list[cb], cb, g->sc, g->a, g->w);
    }
    k_end<<<1, 64, 0, s>>>(cb, g->sc, g->d_sizes, g->d_f, g->d_cap, p->mode, p->k, p->eps_num, p->eps_den);
    KWS_HIP(hipGetLastError());
    if (step % 4 == 0 || known < 4096) {
      PeelScalars h;
      KWS_HIP(hipMemcpyAsync(&h, g->sc, sizeof(h), hipMemcpyDeviceToHost, s));
      KWS_HIP(hipStreamSynchronize(s));
      known = h.s;
      if (h.round + 1 >= g->d_cap) return fail(KWS_EOVERFLOW, "more than %d rounds", g->d_cap - 1);
    }
  }
  k_export<<<grid_for(n, BLOCK, resident), BLOCK, 0, s>>>(n, g->inv, g->rnd_in, g->sc, g->rnd);
  KWS_HIP(hipGetLastError());
  PeelScalars h;
  KWS_HIP(hipMemcpyAsync(&h, g->sc, sizeof(h), hipMemcpyDeviceToHost, s));
  KWS_HIP(hipStreamSynchronize(s));
  // the last round is the one that left nothing (steps enqueued after it did nothing)
  const int32_t round = h.round;
  if (round + 1 > g->d_cap) return fail(KWS_EOVERFLOW, "more than %d rounds", g->d_cap - 1);
  std::vector<int64_t> hs((size_t)round + 1), hf((size_t)round + 1);
  KWS_HIP(hipMemcpyAsync(hs.data(), g->d_sizes, sizeof(int64_t) * hs.size(), hipMemcpyDeviceToHost, s));
  KWS_HIP(hipMemcpyAsync(hf.data(), g->d_f, sizeof(int64_t) * hf.size(), hipMemcpyDeviceToHost, s));
  if (peel_round && n > 0)
    KWS_HIP(hipMemcpyAsync(peel_round, g->rnd, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
  KWS_HIP(hipStreamSynchronize(s));
  const int32_t R = round;
  if ((sizes || f) && R + 1 > cap) return fail(KWS_EOVERFLOW, "%d rounds do not fit cap %d", R, cap);
  if (sizes) std::memcpy(sizes, hs.data(), sizeof(int64_t) * ((size_t)R + 1));
  if (f) std::memcpy(f, hf.data(), sizeof(int64_t) * ((size_t)R + 1));
  sum.rounds = R;
  sum.best = h.best_i < 0 ? 0 : h.best_i;
  sum.best_size = h.best_i < 0 ? 0 : h.best_s;
  sum.best_f = h.best_i < 0 ? 0 : h.best_f;
  sum.incidences = 2 * g->m;   // every vertex is removed once: each edge is visited from both ends
  sum.trims = (int64_t)h.trims;
  evlog.collect(sum);
  sum.steps = (int64_t)R + (int64_t)h.trims;
  if (summary) *summary = sum;
  g->has_run = true;
  return KWS_OK;
}

kws_status kws_dsd_rounds(kws_dsd_graph *g, int32_t *peel_round, const int32_t **device_rounds) {
  using namespace kws;
  clear_error();
  if (!g) return fail(KWS_EINVAL, "null graph");
  if (!g->has_run) return fail(KWS_EINVAL, "no finished peeling run on this graph");
  if (device_rounds) *device_rounds = g->rnd;
  if (peel_round && g->n > 0) {
    KWS_HIP(hipMemcpyAsync(peel_round, g->rnd, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToHost, g->stream));
    KWS_HIP(hipStreamSynchronize(g->stream));
  }
  return KWS_OK;
}

}  // extern "C"
