// Keyword-search pass: bit-parallel bounded multi-source BFS on the reverse
// graph, root filter, scoring, exact top-k and answer-graph extraction.
//
// Lanes. Every (query, keyword) needs one BFS. A lane is one bit of a 64-bit
// mask word; all lanes of a query sit in one word, and queries packed into
// the same word share a lane when they ask for the same keyword with the same
// d_max. Per vertex the pass keeps, for each word:
//   vis    lanes whose BFS has reached the vertex (dist <= current level)
//   fr     lanes that reached it exactly at the current level (two buffers)
//   nxt    lanes arriving at the next level (push target; zero between passes)
//   P_b    bit b of the distance of each reached lane (bit-sliced distances)
// Layout [tile][vertex][T words]: T words of one vertex are contiguous, so
// one neighbour visit gathers 8*T bytes; a tile is one contiguous slab.
//
// Level l expands lanes whose d_max > l, either by push (frontier vertices
// OR their frontier bits into their in-neighbours' nxt with 64-bit atomics)
// or by pull (each vertex that still misses some lane ORs the frontier masks
// of its out-neighbours, no atomics, early exit once all missing lanes are
// found). The choice is made on the device from the frontier statistics of
// the previous level, so the launch sequence never depends on data.
#include <algorithm>
#include <array>
#include <cstring>
#include <unordered_map>

#include "kws_internal.h"

namespace kws {

// ============================================================ device side

struct Pass {
  // sizes
  int32_t n, tiles, Wp, G, D, B, nq, n_lanes;
  int32_t chunks, CH, nhist, hist_lds, te_lds;
  int32_t force_dir;
  float alpha;
  int64_t total_seeds, n_hub, total_slots, total_kd;
  int64_t bin_begin[BIN_COUNT + 1];
  size_t pstride;              // words per plane = tiles * n * T
  // graph
  const int32_t *fwd_ptr, *fwd_col, *rev_ptr, *rev_col, *inv_vtx;
  const int32_t *bin_vtx, *hub_v, *hub_b, *hub_e;
  // state
  uint64_t *vis, *fr0, *fr1, *nxt, *planes;
  int32_t *flist, *flist_eoff;
  // plan
  const uint64_t *act;               // [(D+2) * Wp]
  const int64_t *lane_seed_off;      // [n_lanes + 1]
  const int32_t *lane_seed_begin;    // [n_lanes]
  const int32_t *lane_word, *lane_bit;
  const int32_t *word_q_ptr, *word_q;
  const uint64_t *q_mask;
  const int32_t *q_word, *q_dmax, *q_nk, *q_kcap, *q_hoff, *q_coff, *q_ccap, *q_roff, *q_kdoff,
      *q_eoff, *q_ecap, *q_boff;
  const uint8_t *bits;               // lane bit of each query keyword, keyword order
  const int32_t *q_lane;             // lane id of each query keyword, keyword order
  // zeroed per pass
  uint64_t *zero0; int64_t zero0_words;
  uint64_t *zero1; int64_t zero1_words;
  uint64_t *stats;                   // [(D+1) * 4]: (n_f << 32 | m_f), m_u
  uint64_t *live;                    // [(D+1) * Wp]: lanes with a non-empty frontier
  uint64_t *te;                      // [nq]
  int32_t *cand_cnt, *work_cnt, *hist;
  // per pass scratch
  int32_t *qsel;                     // [nq * 4]: k_eff, s*, need, c_lt
  int4 *work;
  uint64_t *cand;
  // results
  int32_t *r_nroots, *r_roots, *r_scores, *r_ecount;
  uint8_t *r_kwdist;
  int2 *r_edges;
};

__device__ __forceinline__ int pick_dir(const uint64_t *st, float alpha, int force) {
  const uint64_t packed = st[0];
  const uint32_t nf = (uint32_t)(packed >> 32), mf = (uint32_t)packed;
  if (nf == 0) return 0;                       // empty frontier: nothing to expand
  if (force == 1 || force == 2) return force;
  return (double)alpha * (double)mf > (double)st[1] ? 2 : 1;   // 1 push, 2 pull
}

__device__ __forceinline__ uint64_t group_bits(int lane, int S) {
  return S >= 64 ? ~0ull : (((1ull << S) - 1ull) << (lane & ~(S - 1)));
}

__device__ __forceinline__ int32_t wave_incl_scan(int32_t x, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    int32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

// Block-wide exclusive scan of x; *total receives the block sum.
__device__ int32_t block_scan(int32_t x, int32_t *total) {
  __shared__ int32_t s_w[BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t incl = wave_incl_scan(x, lane);
  if (lane == 63) s_w[wid] = incl;
  __syncthreads();
  int32_t base = 0, all = 0;
  for (int w = 0; w < BLOCK / 64; w++) {
    base += w < wid ? s_w[w] : 0;
    all += s_w[w];
  }
  __syncthreads();
  *total = all;
  return base + incl - x;
}

// ---- seed: zero the per-pass counters; OR each lane's bit into nxt of its keyword vertices
template <int T>
__global__ __launch_bounds__(BLOCK) void k_seed(const Pass P) {
  const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, gsz = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = gid; i < P.zero0_words; i += gsz) P.zero0[i] = 0;
  for (int64_t i = gid; i < P.zero1_words; i += gsz) P.zero1[i] = 0;
  for (int64_t i = gid; i < P.total_seeds; i += gsz) {
    int lo = 0, hi = P.n_lanes;               // largest lane with lane_seed_off[lane] <= i
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (P.lane_seed_off[mid] <= i) lo = mid; else hi = mid;
    }
    const int32_t v = P.inv_vtx[P.lane_seed_begin[lo] + (int32_t)(i - P.lane_seed_off[lo])];
    const int word = P.lane_word[lo];
    const size_t idx = ((size_t)(word / T) * P.n + v) * T + (word % T);
    atomicOr((unsigned long long *)&P.nxt[idx], 1ull << P.lane_bit[lo]);
  }
}

// ---- finalize level L -> L+1 (L = -1 turns the seeds into level 0)
// new = nxt & ~vis & act[L+1]; vis |= new; distance planes; next frontier
// buffer; nxt cleared; the statistics that pick the direction of the next
// level. Frontier vertices are compacted into LDS per chunk of FIN_CHUNK
// vertices (wavefront ballot + prefix sums), then one atomic per chunk
// reserves their place in the global list and its in-edge offsets.
constexpr int FIN_CHUNK = 512;

template <int T>
__global__ __launch_bounds__(BLOCK) void k_finalize(const Pass P, int L) {
  extern __shared__ uint64_t s_live[];                    // [Wp]
  __shared__ int32_t s_lv[FIN_CHUNK], s_le[FIN_CHUNK];
  __shared__ int32_t s_wcnt[BLOCK / 64], s_wedge[BLOCK / 64];
  __shared__ int32_t s_cnt, s_edges;
  __shared__ uint64_t s_base;
  const bool first = L < 0;
  const bool last = L + 1 >= P.D;
  constexpr int G = T, VPB = BLOCK / T;   // T threads per vertex, one per word of a tile
  const int tid = threadIdx.x, gl = tid & (G - 1), lane = tid & 63, wid = tid >> 6;
  const uint64_t gmask = group_bits(lane, G);
  const uint64_t *act_new = P.act + (size_t)(L + 1) * P.Wp;
  const uint64_t *act_nn = P.act + (size_t)(L + 2) * P.Wp;
  uint64_t *fr_next = ((L + 1) & 1) ? P.fr1 : P.fr0;
  uint64_t *st = P.stats + (size_t)(L + 1) * 4;
  for (int j = tid; j < P.Wp; j += BLOCK) s_live[j] = 0;
  uint64_t mu_acc = 0;
  const int64_t nchunks = ((int64_t)P.n + FIN_CHUNK - 1) / FIN_CHUNK;
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    if (tid == 0) { s_cnt = 0; s_edges = 0; }
    __syncthreads();
    const int64_t c0 = c * FIN_CHUNK, c1 = min((int64_t)P.n, c0 + FIN_CHUNK);
    for (int64_t vb = c0; vb < c1; vb += VPB) {
      const int64_t v = vb + tid / G;
      const bool valid = v < c1;
      uint64_t anyf = 0, anyneed = 0;
      if (valid) {
        constexpr int TG = 8;   // tiles whose words are loaded before any store
        for (int t0 = 0; t0 < P.tiles; t0 += TG) {
          uint64_t nxv[TG], oldv[TG];
#pragma unroll
          for (int k = 0; k < TG; k++) {
            const size_t idx = ((size_t)(t0 + k) * P.n + v) * T + gl;
            nxv[k] = t0 + k < P.tiles ? P.nxt[idx] : 0ull;
            oldv[k] = (t0 + k < P.tiles && !first) ? P.vis[idx] : 0ull;
          }
#pragma unroll
          for (int k = 0; k < TG; k++) {
            if (t0 + k >= P.tiles) break;
            const int j = (t0 + k) * T + gl;
            const size_t idx = ((size_t)(t0 + k) * P.n + v) * T + gl;
            const uint64_t nx = nxv[k], old = oldv[k];
            const uint64_t fnew = nx & ~old & act_new[j];
            const uint64_t nv = old | fnew;
            if (first) {
              P.vis[idx] = nv;
              for (int b = 0; b < P.B; b++) P.planes[b * P.pstride + idx] = 0;
            } else if (fnew) {
              P.vis[idx] = nv;
              for (int b = 0; b < P.B; b++)
                if (((L + 1) >> b) & 1) P.planes[b * P.pstride + idx] |= fnew;
            }
            if (!last) {
              fr_next[idx] = fnew;
              if (fnew) atomicOr((unsigned long long *)&s_live[j], fnew);
              anyneed |= act_nn[j] & ~nv;
            }
            if (nx) P.nxt[idx] = 0;
            anyf |= fnew;
          }
        }
      }
      const bool fflag = (__ballot(anyf != 0) & gmask) != 0;
      const bool nflag = (__ballot(anyneed != 0) & gmask) != 0;
      const bool take = valid && gl == 0 && fflag;
      if (valid && gl == 0 && nflag) mu_acc += (uint64_t)(P.fwd_ptr[v + 1] - P.fwd_ptr[v]);
      const int32_t indeg = take ? P.rev_ptr[v + 1] - P.rev_ptr[v] : 0;
      const uint64_t bal = __ballot(take);
      const int32_t wpre = __popcll(bal & ((1ull << lane) - 1ull));
      const int32_t eincl = wave_incl_scan(indeg, lane);
      if (lane == 63) { s_wcnt[wid] = __popcll(bal); s_wedge[wid] = eincl; }
      __syncthreads();
      if (take) {
        int32_t cpre = s_cnt, epre = s_edges;
        for (int w = 0; w < wid; w++) { cpre += s_wcnt[w]; epre += s_wedge[w]; }
        s_lv[cpre + wpre] = (int32_t)v;
        s_le[cpre + wpre] = epre + eincl - indeg;
      }
      __syncthreads();
      if (tid == 0)
        for (int w = 0; w < BLOCK / 64; w++) { s_cnt += s_wcnt[w]; s_edges += s_wedge[w]; }
      __syncthreads();
    }
    if (tid == 0)
      s_base = s_cnt ? atomicAdd((unsigned long long *)&st[0],
                                 (unsigned long long)(((uint64_t)s_cnt << 32) | (uint32_t)s_edges))
                     : 0ull;
    __syncthreads();
    if (!last) {
      const int32_t bc = (int32_t)(s_base >> 32), be = (int32_t)(uint32_t)s_base;
      for (int i = tid; i < s_cnt; i += BLOCK) {
        P.flist[bc + i] = s_lv[i];
        P.flist_eoff[bc + i] = be + s_le[i];
      }
    }
    __syncthreads();
  }
  if (!last) {
    __syncthreads();
    for (int j = tid; j < P.Wp; j += BLOCK)
      if (s_live[j]) atomicOr((unsigned long long *)&P.live[(size_t)(L + 1) * P.Wp + j], s_live[j]);
    for (int off = 32; off > 0; off >>= 1) mu_acc += __shfl_xor(mu_acc, off);
    if (lane == 0 && mu_acc) atomicAdd((unsigned long long *)&st[1], (unsigned long long)mu_acc);
  }
}

// ---- push: every frontier in-edge (p -> v) ORs v's frontier lanes into nxt[p]
// Wq threads per edge cover the words (power of two, <= 64).
template <int T>
__global__ __launch_bounds__(BLOCK) void k_push(const Pass P, int L, int Wq) {
  const uint64_t *st = P.stats + (size_t)L * 4;
  if (pick_dir(st, P.alpha, P.force_dir) != 1) return;
  const int32_t nf = (int32_t)(st[0] >> 32);
  const int64_t mf = (int64_t)(uint32_t)st[0];
  const int EPB = BLOCK / Wq;
  const int tid = threadIdx.x, wq = tid & (Wq - 1), es = tid / Wq;
  const uint64_t *fr = (L & 1) ? P.fr1 : P.fr0;
  const uint64_t *act = P.act + (size_t)(L + 1) * P.Wp;
  const uint64_t *live = P.live + (size_t)L * P.Wp;
  __shared__ int32_t s_j;
  for (int64_t eb = (int64_t)blockIdx.x * EPB; eb < mf; eb += (int64_t)gridDim.x * EPB) {
    if (tid == 0) {
      int32_t lo = 0, hi = nf;                // largest j with flist_eoff[j] <= eb
      while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (P.flist_eoff[mid] <= eb) lo = mid; else hi = mid;
      }
      s_j = lo;
    }
    __syncthreads();
    int32_t j = s_j;
    __syncthreads();
    const int64_t e = eb + es;
    if (e >= mf) continue;
    while (j + 1 < nf && P.flist_eoff[j + 1] <= e) j++;
    const int32_t v = P.flist[j];
    const int32_t p = P.rev_col[P.rev_ptr[v] + (int32_t)(e - P.flist_eoff[j])];
    for (int word = wq; word < P.Wp; word += Wq) {
      const size_t tb = (size_t)(word / T) * P.n * T;
      const int w = word % T;
      uint64_t f = fr[tb + (size_t)v * T + w] & act[word] & live[word];
      if (!f) continue;
      f &= ~P.vis[tb + (size_t)p * T + w];
      if (f) atomicOr((unsigned long long *)&P.nxt[tb + (size_t)p * T + w], f);
    }
  }
}

// ---- pull: a group of S = T*E threads owns one row (or one hub chunk);
// thread (e, w) ORs word w of the frontier mask of every E-th out-neighbour.
// Early exit once the group has found every lane the vertex still misses.
template <int T, int S, bool SEG>
__device__ __forceinline__ void pull_rows(const Pass &P, int L, const int32_t *items, int64_t n_items, int tile,
                                          int bb, int bpt) {
  constexpr int E = S / T, GPB = BLOCK / S, U = 4;
  const int tid = threadIdx.x, gl = tid % S, w = gl % T, eo = gl / T, lane = tid & 63;
  const uint64_t gmask = group_bits(lane, S);
  const size_t tb = (size_t)tile * P.n * T;
  const uint64_t *fr = ((L & 1) ? P.fr1 : P.fr0) + tb;
  const uint64_t *vis = P.vis + tb;
  uint64_t *nxt = P.nxt + tb;
  const int word = tile * T + w;
  const uint64_t actw = P.act[(size_t)(L + 1) * P.Wp + word] & P.live[(size_t)L * P.Wp + word];
  const int32_t *col = P.fwd_col;
  for (int64_t it = (int64_t)bb * GPB + tid / S; it < n_items; it += (int64_t)bpt * GPB) {
    int32_t v, eb, ee;
    if (SEG) {
      v = P.hub_v[it]; eb = P.hub_b[it]; ee = P.hub_e[it];
    } else {
      v = items[it]; eb = P.fwd_ptr[v]; ee = P.fwd_ptr[v + 1];
    }
    const uint64_t need = actw & ~vis[(size_t)v * T + w];
    if ((__ballot(need != 0) & gmask) == 0) continue;
    uint64_t acc = 0;
    for (int32_t e0 = eb; e0 < ee; e0 += E * U) {
      int32_t x[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int32_t e = e0 + u * E + eo;
        x[u] = e < ee ? col[e] : -1;
      }
#pragma unroll
      for (int u = 0; u < U; u++)
        if (x[u] >= 0) acc |= fr[(size_t)x[u] * T + w];
      uint64_t r = acc;
#pragma unroll
      for (int off = T; off < S; off <<= 1) r |= __shfl_xor(r, off);
      if ((__ballot((r & need) != need) & gmask) == 0) break;
    }
#pragma unroll
    for (int off = T; off < S; off <<= 1) acc |= __shfl_xor(acc, off);
    acc &= need;
    if (eo == 0 && acc) {
      if (SEG) atomicOr((unsigned long long *)&nxt[(size_t)v * T + w], acc);
      else nxt[(size_t)v * T + w] = acc;
    }
  }
}

// One launch covers every degree bin: blocks [boff[b], boff[b+1]) serve bin b
// (b = 3 is the hub chunks), tiles x blocks-per-tile inside each range.
struct PullGrid { int32_t boff[BIN_COUNT + 2]; };

template <int T>
__global__ __launch_bounds__(BLOCK) void k_pull(const Pass P, int L, const PullGrid pg) {
  if (pick_dir(P.stats + (size_t)L * 4, P.alpha, P.force_dir) != 2) return;
  constexpr int S_SMALL = T, S_MED = (8 * T < 64 ? 8 * T : 64);
  const int bid = blockIdx.x;
  if (bid >= pg.boff[BIN_COUNT + 1]) return;   // the grid has one block even when every bin is empty
  int b = 0;
  while (b < BIN_COUNT && bid >= pg.boff[b + 1]) b++;
  const int nblk = pg.boff[b + 1] - pg.boff[b];
  const int bpt = nblk / P.tiles, lb = bid - pg.boff[b];
  const int tile = lb / bpt, bb = lb % bpt;
  if (tile >= P.tiles) return;
  if (b == BIN_COUNT) {
    pull_rows<T, 64, true>(P, L, nullptr, P.n_hub, tile, bb, bpt);
    return;
  }
  const int32_t *items = P.bin_vtx + P.bin_begin[b];
  const int64_t n_items = P.bin_begin[b + 1] - P.bin_begin[b];
  if (b == BIN_SMALL) pull_rows<T, S_SMALL, false>(P, L, items, n_items, tile, bb, bpt);
  else if (b == BIN_MEDIUM) pull_rows<T, S_MED, false>(P, L, items, n_items, tile, bb, bpt);
  else pull_rows<T, 64, false>(P, L, items, n_items, tile, bb, bpt);
}

// ---- score: per vertex and query, root test, score histogram per chunk and
// the scanned-edge count te (in-degree of every vertex each lane expanded).
// Each thread holds SC_R vertices; a wavefront walks the words and their
// queries in lockstep, so histogram updates are aggregated per distinct
// score value and te is reduced across the wavefront once per query.
constexpr int SC_R = 2;

template <int T>
__global__ __launch_bounds__(BLOCK) void k_score(const Pass P) {
  extern __shared__ uint64_t s_dyn[];
  uint64_t *s_te = s_dyn;
  int32_t *s_hist = (int32_t *)(s_dyn + (P.te_lds ? P.nq : 0));
  const int tid = threadIdx.x, lane = tid & 63;
  const int split = (P.CH + BLOCK * SC_R - 1) / (BLOCK * SC_R);
  if (P.te_lds)
    for (int i = tid; i < P.nq; i += BLOCK) s_te[i] = 0;
  for (int64_t bid = blockIdx.x; bid < (int64_t)P.chunks * split; bid += gridDim.x) {
    const int c = (int)(bid / split), part = (int)(bid % split);
    if (P.hist_lds)
      for (int i = tid; i < P.nhist; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    int32_t *hist = P.hist_lds ? s_hist : P.hist + (size_t)c * P.nhist;
    const int64_t cend = min((int64_t)P.n, (int64_t)(c + 1) * P.CH);
    const int64_t v0 = (int64_t)c * P.CH + (int64_t)part * BLOCK * SC_R;
    int64_t vv[SC_R];
    uint64_t indeg[SC_R];
#pragma unroll
    for (int r = 0; r < SC_R; r++) {
      vv[r] = v0 + r * BLOCK + tid;
      indeg[r] = vv[r] < cend ? (uint64_t)(P.rev_ptr[vv[r] + 1] - P.rev_ptr[vv[r]]) : 0ull;
    }
    for (int j = 0; j < P.Wp; j++) {
      const int qb = P.word_q_ptr[j], qe = P.word_q_ptr[j + 1];
      if (qb == qe) continue;
      const size_t base = (size_t)(j / T) * P.n * T + (j % T);
      uint64_t vis[SC_R], pl[SC_R][4];
      bool any = false;
#pragma unroll
      for (int r = 0; r < SC_R; r++) {
        vis[r] = vv[r] < cend ? P.vis[base + (size_t)vv[r] * T] : 0ull;
        for (int b = 0; b < 4; b++)
          pl[r][b] = (b < P.B && vis[r]) ? P.planes[b * P.pstride + base + (size_t)vv[r] * T] : 0ull;
        any |= vis[r] != 0;
      }
      if (__ballot(any) == 0) continue;
      for (int qi = qb; qi < qe; qi++) {
        const int q = P.word_q[qi];
        const uint64_t m = P.q_mask[q];
        const int dq = P.q_dmax[q], hq = P.q_hoff[q];
        uint64_t t = 0;
#pragma unroll
        for (int r = 0; r < SC_R; r++) {
          const uint64_t x = vis[r] & m;
          uint64_t eq = x;
          for (int b = 0; b < P.B; b++) eq &= ((dq >> b) & 1) ? pl[r][b] : ~pl[r][b];
          t += (uint64_t)(__popcll(x) - __popcll(eq)) * indeg[r];
          const bool root = x == m;
          int sc = 0;
          if (root)
            for (int b = 0; b < P.B; b++) sc += __popcll(pl[r][b] & m) << b;
          uint64_t pend = __ballot(root);
          while (pend) {
            const int leader = __ffsll((long long)pend) - 1;
            const int sv = __shfl(sc, leader);
            const uint64_t same = __ballot(root && sc == sv);
            if (lane == leader) atomicAdd(&hist[hq + sv], (int)__popcll(same));
            pend &= ~same;
          }
        }
        if (__ballot(t != 0)) {
          for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
          if (lane == 0) {
            if (P.te_lds) atomicAdd((unsigned long long *)&s_te[q], (unsigned long long)t);
            else atomicAdd((unsigned long long *)&P.te[q], (unsigned long long)t);
          }
        }
      }
    }
    __syncthreads();
    if (P.hist_lds)
      for (int i = tid; i < P.nhist; i += BLOCK)
        if (s_hist[i]) atomicAdd(&P.hist[(size_t)c * P.nhist + i], s_hist[i]);
    __syncthreads();
  }
  if (P.te_lds) {
    __syncthreads();
    for (int i = tid; i < P.nq; i += BLOCK)
      if (s_te[i]) atomicAdd((unsigned long long *)&P.te[i], (unsigned long long)s_te[i]);
  }
}

// ---- threshold: per query, the score s* of the k-th root, how many ties at
// s* to take, and one work item per chunk that holds a selected root.
__global__ __launch_bounds__(BLOCK) void k_threshold(const Pass P) {
  __shared__ int32_t tot[KWS_MAX_KW * KWS_MAX_DMAX + 1];
  __shared__ int32_t s_sel[4];
  const int tid = threadIdx.x;
  for (int q = blockIdx.x; q < P.nq; q += gridDim.x) {
    const int S1 = P.q_nk[q] * P.q_dmax[q] + 1, hoff = P.q_hoff[q];
    for (int s = tid; s < S1; s += BLOCK) tot[s] = 0;
    __syncthreads();
    for (int64_t i = tid; i < (int64_t)P.chunks * S1; i += BLOCK) {
      const int c = (int)(i / S1), s = (int)(i % S1);
      const int32_t h = P.hist[(size_t)c * P.nhist + hoff + s];
      if (h) atomicAdd(&tot[s], h);
    }
    __syncthreads();
    if (tid == 0) {
      int64_t total = 0;
      for (int s = 0; s < S1; s++) total += tot[s];
      const int32_t keff = (int32_t)min((int64_t)P.q_kcap[q], total);
      int32_t sstar = -1, need = 0, clt = 0, cum = 0;
      if (keff > 0)
        for (int s = 0; s < S1; s++) {
          if (cum + tot[s] >= keff) { sstar = s; clt = cum; need = keff - cum; break; }
          cum += tot[s];
        }
      s_sel[0] = keff; s_sel[1] = sstar; s_sel[2] = need; s_sel[3] = clt;
      P.qsel[q * 4 + 0] = keff; P.qsel[q * 4 + 1] = sstar;
      P.qsel[q * 4 + 2] = need; P.qsel[q * 4 + 3] = clt;
      P.r_nroots[q] = keff;
    }
    __syncthreads();
    const int32_t keff = s_sel[0], sstar = s_sel[1], need = s_sel[2];
    if (keff > 0) {
      int32_t carry = 0;
      for (int base = 0; base < P.chunks; base += BLOCK) {
        const int c = base + tid;
        int32_t t = 0, lt = 0;
        if (c < P.chunks) {
          const int32_t *h = P.hist + (size_t)c * P.nhist + hoff;
          t = h[sstar];
          for (int s = 0; s < sstar; s++) lt += h[s];
        }
        int32_t btot;
        const int32_t ex = block_scan(t, &btot) + carry;
        carry += btot;
        if (c < P.chunks && (lt > 0 || (t > 0 && ex < need))) {
          const int32_t pos = atomicAdd(P.work_cnt, 1);
          P.work[pos] = make_int4(q, c, ex, lt);
        }
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int lane_dist(const Pass &P, size_t idx, int bit) {
  int d = 0;
  for (int b = 0; b < P.B; b++) d |= (int)((P.planes[b * P.pstride + idx] >> bit) & 1ull) << b;
  return d;
}

// ---- select: scan one chunk for one query in vertex order; keep every root
// below s* and the first `need` ties overall (ranked across chunks).
template <int T>
__global__ __launch_bounds__(BLOCK) void k_select(const Pass P) {
  const int tid = threadIdx.x;
  const int n_items = *P.work_cnt;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 wk = P.work[it];
    const int q = wk.x, c = wk.y, lt_c = wk.w;
    const int32_t sstar = P.qsel[q * 4 + 1], need = P.qsel[q * 4 + 2];
    const int word = P.q_word[q];
    const uint64_t m = P.q_mask[q];
    const size_t tb = (size_t)(word / T) * P.n * T;
    const int w = word % T;
    int32_t ties = wk.z, lts = 0;
    const int64_t v0 = (int64_t)c * P.CH, v1 = min((int64_t)P.n, v0 + P.CH);
    for (int64_t vb = v0; vb < v1; vb += BLOCK) {
      const int64_t v = vb + tid;
      bool lt = false, tie = false;
      int s = 0;
      if (v < v1) {
        const size_t idx = tb + (size_t)v * T + w;
        if ((P.vis[idx] & m) == m) {
          for (int b = 0; b < P.B; b++) s += __popcll(P.planes[b * P.pstride + idx] & m) << b;
          lt = s < sstar;
          tie = s == sstar;
        }
      }
      int32_t ntie, nlt;
      const int32_t rank = block_scan(tie ? 1 : 0, &ntie) + ties;
      block_scan(lt ? 1 : 0, &nlt);
      if (lt || (tie && rank < need)) {
        const int32_t pos = atomicAdd(&P.cand_cnt[q], 1);
        P.cand[P.q_coff[q] + pos] = ((uint64_t)(uint32_t)s << 32) | (uint64_t)(uint32_t)v;
      }
      ties += ntie;
      lts += nlt;
      if (lts >= lt_c && ties >= need) break;
    }
    __syncthreads();
  }
}

// ---- finish: order each query's candidates by (score, id); write roots,
// scores and the per-keyword distances.
template <int T>
__global__ __launch_bounds__(BLOCK) void k_finish(const Pass P) {
  constexpr int LDS_SORT = 2048;
  __shared__ uint64_t s_key[LDS_SORT];
  const int tid = threadIdx.x;
  for (int q = blockIdx.x; q < P.nq; q += gridDim.x) {
    const int32_t keff = P.qsel[q * 4 + 0];
    if (keff == 0) continue;
    uint64_t *g = P.cand + P.q_coff[q];
    int N = 1;
    while (N < keff) N <<= 1;
    uint64_t *x = N <= LDS_SORT ? s_key : g;
    for (int i = tid; i < N; i += BLOCK) x[i] = i < keff ? g[i] : ~0ull;
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < N; i += BLOCK) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const uint64_t a = x[i], b = x[ixj];
            if ((a > b) == ((i & k) == 0)) { x[i] = b; x[ixj] = a; }
          }
        }
        __syncthreads();
      }
    const int word = P.q_word[q], w = word % T, nk = P.q_nk[q];
    const size_t tb = (size_t)(word / T) * P.n * T;
    const int roff = P.q_roff[q], kdoff = P.q_kdoff[q], boff = P.q_boff[q];
    for (int i = tid; i < keff; i += BLOCK) {
      const uint64_t key = x[i];
      const int32_t v = (int32_t)(uint32_t)key;
      P.r_roots[roff + i] = v;
      P.r_scores[roff + i] = (int32_t)(key >> 32);
      const size_t idx = tb + (size_t)v * T + w;
      for (int j = 0; j < nk; j++) P.r_kwdist[kdoff + (size_t)i * nk + j] = (uint8_t)lane_dist(P, idx, P.bits[boff + j]);
    }
    __syncthreads();
  }
}

// ---- answer: one wave per (query, root, keyword) walks from the root to
// the smallest-id out-neighbour one hop closer, writing the path into the
// keyword's segment of the root's edge slot; then one wave per (query, root)
// merges the segments: sort, drop repeats.
template <int T>
__global__ __launch_bounds__(BLOCK) void k_answer(const Pass P) {
  constexpr int WAVES = BLOCK / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t waves = (int64_t)gridDim.x * WAVES;
  for (int64_t item = (int64_t)blockIdx.x * WAVES + wid; item < P.total_kd; item += waves) {
    int lo = 0, hi = P.nq;                      // query owning this (root, keyword) item
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (P.q_kdoff[mid] <= item) lo = mid; else hi = mid;
    }
    const int q = lo, nk = P.q_nk[q];
    const int rel = (int)(item - P.q_kdoff[q]), i = rel / nk, j = rel % nk;
    if (i >= P.qsel[q * 4 + 0]) continue;
    const int32_t r = P.r_roots[P.q_roff[q] + i];
    int d = P.r_kwdist[item];
    const int word = P.q_word[q], w = word % T, bit = P.bits[P.q_boff[q] + j];
    const size_t tb = (size_t)(word / T) * P.n * T;
    int2 *out = P.r_edges + P.q_eoff[q] + (size_t)i * P.q_ecap[q] + (size_t)j * P.q_dmax[q];
    int32_t x = r;
    int h = 0;
    const int lid = P.q_lane[P.q_boff[q] + j];
    while (d > 0) {
      int32_t best = 0x7fffffff;
      const int32_t e0 = P.fwd_ptr[x], e1 = P.fwd_ptr[x + 1];
      const int64_t ns = P.lane_seed_off[lid + 1] - P.lane_seed_off[lid];
      if (d == 1 && ns * 4 < (int64_t)(e1 - e0)) {
        // last hop: the keyword's vertices are few compared with the row, so
        // look each of them up in the sorted row and keep the smallest hit
        const int32_t *seeds = P.inv_vtx + P.lane_seed_begin[lid];
        int32_t mine = 0x7fffffff;
        for (int64_t k = lane; k < ns; k += 64) {
          const int32_t v = seeds[k];
          int32_t lo = e0, hi = e1;
          while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (P.fwd_col[mid] < v) lo = mid + 1; else hi = mid;
          }
          if (lo < e1 && P.fwd_col[lo] == v) mine = min(mine, v);
        }
        for (int off = 32; off > 0; off >>= 1) mine = min(mine, __shfl_xor(mine, off));
        best = mine;
      } else {
        // rows are sorted by neighbour id, so the first qualifying neighbour
        // in row order is the smallest-id one; four chunks of 64 per round
        constexpr int U = 4;
        for (int32_t eb = e0; eb < e1 && best == 0x7fffffff; eb += 64 * U) {
          int32_t y[U];
          bool ok[U];
#pragma unroll
          for (int u = 0; u < U; u++) {
            const int32_t e = eb + u * 64 + lane;
            y[u] = e < e1 ? P.fwd_col[e] : -1;
          }
#pragma unroll
          for (int u = 0; u < U; u++)
            ok[u] = y[u] >= 0 && ((P.vis[tb + (size_t)y[u] * T + w] >> bit) & 1ull);
#pragma unroll
          for (int u = 0; u < U; u++)
            if (ok[u]) ok[u] = lane_dist(P, tb + (size_t)y[u] * T + w, bit) == d - 1;
#pragma unroll
          for (int u = 0; u < U; u++) {
            const uint64_t bal = __ballot(ok[u]);
            if (bal && best == 0x7fffffff) best = __shfl(y[u], __ffsll((long long)bal) - 1);
          }
        }
      }
      if (best == 0x7fffffff || h >= P.q_dmax[q]) break;   // cannot happen for a BFS-consistent state
      if (lane == 0) out[h] = make_int2(x, best);
      h++;
      x = best;
      d--;
    }
  }
}

template <int T>
__global__ __launch_bounds__(BLOCK) void k_answer_merge(const Pass P) {
  constexpr int WAVES = BLOCK / 64, ECAP = KWS_MAX_KW * KWS_MAX_DMAX;
  __shared__ uint64_t s_e[WAVES][ECAP];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint64_t *eb = s_e[wid];
  const int64_t waves = (int64_t)gridDim.x * WAVES;
  for (int64_t slot = (int64_t)blockIdx.x * WAVES + wid; slot < P.total_slots; slot += waves) {
    if (lane != 0) continue;
    int lo = 0, hi = P.nq;                      // query owning this slot
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (P.q_roff[mid] <= slot) lo = mid; else hi = mid;
    }
    const int q = lo, i = (int)(slot - P.q_roff[q]);
    if (i >= P.qsel[q * 4 + 0]) continue;
    const int nk = P.q_nk[q], dm = P.q_dmax[q];
    int2 *seg = P.r_edges + P.q_eoff[q] + (size_t)i * P.q_ecap[q];
    const uint8_t *kd = P.r_kwdist + P.q_kdoff[q] + (size_t)i * nk;
    int ne = 0;
    for (int j = 0; j < nk; j++)
      for (int h = 0; h < kd[j] && h < dm; h++) {
        const int2 e = seg[j * dm + h];
        eb[ne++] = ((uint64_t)(uint32_t)e.x << 32) | (uint32_t)e.y;
      }
    for (int a = 1; a < ne; a++) {             // insertion sort, then drop repeats
      const uint64_t key = eb[a];
      int b = a - 1;
      while (b >= 0 && eb[b] > key) { eb[b + 1] = eb[b]; b--; }
      eb[b + 1] = key;
    }
    int u = 0;
    for (int a = 0; a < ne; a++) {
      if (a > 0 && eb[a] == eb[a - 1]) continue;
      seg[u++] = make_int2((int32_t)(eb[a] >> 32), (int32_t)(uint32_t)eb[a]);
    }
    P.r_ecount[slot] = u;
  }
}

// ---- export one lane's distances (verification entry point)
template <int T>
__global__ __launch_bounds__(BLOCK) void k_export(const Pass P, uint8_t *out) {
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < P.n; v += (int64_t)gridDim.x * BLOCK) {
    const size_t idx = (size_t)v * T;
    out[v] = (P.vis[idx] & 1ull) ? (uint8_t)lane_dist(P, idx, 0) : (uint8_t)KWS_DIST_INF;
  }
}

// ============================================================ host side

namespace {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int pow2ceil(int x) { int p = 1; while (p < x) p <<= 1; return p; }
inline unsigned clamp_grid(int64_t blocks) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 1 << 16));
}

struct QIn {
  int32_t nk, dmax, k;
  int32_t kw[KWS_MAX_KW];
};

struct LaneInfo { int32_t kw, dmax, word, bit; };

// Lanes of one pass and where each query sits.
struct Packing {
  std::vector<LaneInfo> lanes;
  std::vector<int32_t> word_used;
  std::vector<int32_t> q_word;
  std::vector<std::array<uint8_t, KWS_MAX_KW>> q_bits;
  std::vector<std::array<int32_t, KWS_MAX_KW>> q_lanes;
  std::vector<uint64_t> q_mask;
  int32_t lane_slots = 0;
};

// Puts queries [qa, qb) into words. A query needs nk lanes in one word; with
// sharing, a keyword already present in that word with the same d_max is
// reused. Among words with room, the one that shares most is chosen (first
// on ties); otherwise a new word is opened.
void pack(const std::vector<QIn> &qs, int qa, int qb, bool share, Packing &pk) {
  pk = Packing();
  std::unordered_map<uint64_t, std::vector<std::array<int32_t, 3>>> where;   // (kw,d) -> (word, bit, lane)
  std::vector<int32_t> shared_cnt;
  for (int q = qa; q < qb; q++) {
    const QIn &Q = qs[q];
    int best = -1, best_sh = -1;
    if (share) {
      shared_cnt.assign(pk.word_used.size(), 0);
      for (int j = 0; j < Q.nk; j++) {
        auto it = where.find(((uint64_t)(uint32_t)Q.kw[j] << 8) | (uint64_t)Q.dmax);
        if (it != where.end())
          for (auto &wb : it->second) shared_cnt[wb[0]]++;
      }
      for (size_t w = 0; w < pk.word_used.size(); w++) {
        const int need = Q.nk - shared_cnt[w];
        if (pk.word_used[w] + need <= 64 && shared_cnt[w] > best_sh) { best = (int)w; best_sh = shared_cnt[w]; }
      }
    } else {
      for (size_t w = 0; w < pk.word_used.size(); w++)
        if (pk.word_used[w] + Q.nk <= 64) { best = (int)w; break; }
    }
    if (best < 0) {
      best = (int)pk.word_used.size();
      pk.word_used.push_back(0);
    }
    std::array<uint8_t, KWS_MAX_KW> bits{};
    std::array<int32_t, KWS_MAX_KW> lids{};
    uint64_t mask = 0;
    for (int j = 0; j < Q.nk; j++) {
      const uint64_t key = ((uint64_t)(uint32_t)Q.kw[j] << 8) | (uint64_t)Q.dmax;
      int bit = -1, lid = -1;
      if (share) {
        auto it = where.find(key);
        if (it != where.end())
          for (auto &wb : it->second)
            if (wb[0] == best) { bit = wb[1]; lid = wb[2]; break; }
      }
      if (bit < 0) {
        bit = pk.word_used[best]++;
        lid = (int)pk.lanes.size();
        pk.lanes.push_back({Q.kw[j], Q.dmax, best, bit});
        where[key].push_back({best, bit, lid});
      }
      bits[j] = (uint8_t)bit;
      lids[j] = lid;
      mask |= 1ull << bit;
    }
    pk.q_word.push_back(best);
    pk.q_bits.push_back(bits);
    pk.q_lanes.push_back(lids);
    pk.q_mask.push_back(mask);
    pk.lane_slots += Q.nk;
  }
}

// Byte layout helper for the plan and result buffers.
struct Layout {
  size_t size = 0;
  size_t add(size_t bytes, size_t align = 256) {
    size = align_up(size, align);
    size_t off = size;
    size += bytes;
    return off;
  }
};

kws_status launch_check(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(KWS_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
  return KWS_OK;
}

struct Timer {
  Profiler &p;
  hipStream_t s;
  int cls;
  hipEvent_t a = nullptr;
  Timer(Profiler &p_, hipStream_t s_, int c) : p(p_), s(s_), cls(c) { p.begin(cls, s, &a); }
  ~Timer() { p.end(cls, s, a); }
};

template <int T>
kws_status run_pass_kernels(kws_graph *g, const Pass &P, int Wq, bool capture_ok) {
  hipStream_t s = g->stream;
  Profiler &prof = g->prof;
  const int64_t seed_items = std::max<int64_t>(P.total_seeds, std::max(P.zero0_words, P.zero1_words));
  {
    Timer t(prof, s, KC_SEED);
    k_seed<T><<<clamp_grid((seed_items + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(P);
  }
  KWS_TRY(launch_check("seed"));
  const unsigned fin_grid = clamp_grid(std::min<int64_t>(((int64_t)P.n + FIN_CHUNK - 1) / FIN_CHUNK, 8192));
  const size_t fin_lds = sizeof(uint64_t) * (size_t)P.Wp;
  {
    Timer t(prof, s, KC_FINALIZE);
    k_finalize<T><<<fin_grid, BLOCK, fin_lds, s>>>(P, -1);
  }
  KWS_TRY(launch_check("finalize"));
  constexpr int S_SMALL = T, S_MED = (8 * T < 64 ? 8 * T : 64);
  PullGrid pg;
  {
    const int sizes[BIN_COUNT + 1] = {S_SMALL, S_MED, 64, 64};
    pg.boff[0] = 0;
    for (int b = 0; b <= BIN_COUNT; b++) {
      const int64_t items = b < BIN_COUNT ? P.bin_begin[b + 1] - P.bin_begin[b] : P.n_hub;
      const int64_t gpb = BLOCK / sizes[b];
      const int64_t bpt = items ? std::min<int64_t>((items + gpb - 1) / gpb, 16384 / P.tiles + 1) : 0;
      pg.boff[b + 1] = pg.boff[b] + (int32_t)(bpt * P.tiles);
    }
  }
  const unsigned pg_total = (unsigned)std::max(1, pg.boff[BIN_COUNT + 1]);
  for (int L = 0; L < P.D; L++) {
    {
      Timer t(prof, s, KC_PUSH);
      k_push<T><<<2048, BLOCK, 0, s>>>(P, L, Wq);
    }
    KWS_TRY(launch_check("push"));
    {
      Timer t(prof, s, KC_PULL);
      k_pull<T><<<pg_total, BLOCK, 0, s>>>(P, L, pg);
    }
    KWS_TRY(launch_check("pull"));
    {
      Timer t(prof, s, KC_FINALIZE);
      k_finalize<T><<<fin_grid, BLOCK, fin_lds, s>>>(P, L);
    }
    KWS_TRY(launch_check("finalize"));
  }
  {
    Timer t(prof, s, KC_SCORE);
    const size_t lds = (P.te_lds ? sizeof(uint64_t) * P.nq : 0) + (P.hist_lds ? sizeof(int32_t) * P.nhist : 0);
    const int64_t split = (P.CH + BLOCK * SC_R - 1) / (BLOCK * SC_R);
    k_score<T><<<clamp_grid(P.chunks * split), BLOCK, lds, s>>>(P);
  }
  KWS_TRY(launch_check("score"));
  {
    Timer t(prof, s, KC_THRESHOLD);
    k_threshold<<<clamp_grid(P.nq), BLOCK, 0, s>>>(P);
  }
  KWS_TRY(launch_check("threshold"));
  {
    Timer t(prof, s, KC_SELECT);
    k_select<T><<<2048, BLOCK, 0, s>>>(P);
  }
  KWS_TRY(launch_check("select"));
  {
    Timer t(prof, s, KC_FINISH);
    k_finish<T><<<clamp_grid(P.nq), BLOCK, 0, s>>>(P);
  }
  KWS_TRY(launch_check("finish"));
  {
    Timer t(prof, s, KC_ANSWER);
    const int64_t waves = BLOCK / 64;
    k_answer<T><<<clamp_grid((P.total_kd + waves - 1) / waves), BLOCK, 0, s>>>(P);
    k_answer_merge<T><<<clamp_grid((P.total_slots + waves - 1) / waves), BLOCK, 0, s>>>(P);
  }
  KWS_TRY(launch_check("answer"));
  (void)capture_ok;
  return KWS_OK;
}

kws_status run_kernels(kws_graph *g, const Pass &P, int T, int Wq) {
  switch (T) {
    case 1: return run_pass_kernels<1>(g, P, Wq, true);
    case 2: return run_pass_kernels<2>(g, P, Wq, true);
    case 4: return run_pass_kernels<4>(g, P, Wq, true);
    case 8: return run_pass_kernels<8>(g, P, Wq, true);
    case 16: return run_pass_kernels<16>(g, P, Wq, true);
  }
  return fail(KWS_EINVAL, "tile_words must be 1, 2, 4, 8 or 16");
}

// Launches the pass through a cached hipGraph keyed by every launch argument.
kws_status run_graph(kws_graph *g, const Pass &P, int T, int Wq) {
  std::vector<uint8_t> key(sizeof(Pass) + 2 * sizeof(int));
  std::memcpy(key.data(), &P, sizeof(Pass));
  std::memcpy(key.data() + sizeof(Pass), &T, sizeof(int));
  std::memcpy(key.data() + sizeof(Pass) + sizeof(int), &Wq, sizeof(int));
  for (auto &e : g->graphs)
    if (e.key == key) {
      KWS_HIP(hipGraphLaunch(e.exec, g->stream));
      return KWS_OK;
    }
  hipGraph_t graph = nullptr;
  KWS_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
  kws_status st = run_kernels(g, P, T, Wq);
  hipError_t e = hipStreamEndCapture(g->stream, &graph);
  if (st != KWS_OK) { if (graph) (void)hipGraphDestroy(graph); return st; }
  if (e != hipSuccess) return fail(KWS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(KWS_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
  if (g->graphs.size() >= 16) {
    (void)hipGraphExecDestroy(g->graphs.front().exec);
    g->graphs.erase(g->graphs.begin());
  }
  g->graphs.push_back({key, exec});
  KWS_HIP(hipGraphLaunch(exec, g->stream));
  return KWS_OK;
}

__global__ void k_fill_u64(uint64_t *p, size_t count) {
  for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += (size_t)gridDim.x * BLOCK) p[i] = 0;
}

// Grows the per-vertex state to hold `words` words per vertex. nxt must be
// zero between passes, so a fresh nxt is cleared.
kws_status ensure_state(kws_graph *g, size_t words_per_array) {
  Engine &E = g->eng;
  if (words_per_array <= E.state_words) return KWS_OK;
  const size_t b = words_per_array * sizeof(uint64_t);
  E.vis.release(); E.fr0.release(); E.fr1.release(); E.nxt.release(); E.planes.release();
  E.state_words = 0;
  KWS_TRY(E.vis.ensure(b, "vis"));
  KWS_TRY(E.fr0.ensure(b, "frontier"));
  KWS_TRY(E.fr1.ensure(b, "frontier"));
  KWS_TRY(E.nxt.ensure(b, "next"));
  KWS_TRY(E.planes.ensure(4 * b, "distance planes"));
  k_fill_u64<<<4096, BLOCK, 0, g->stream>>>(E.nxt.as<uint64_t>(), words_per_array);
  KWS_TRY(launch_check("fill"));
  E.state_words = words_per_array;
  return KWS_OK;
}

struct PassOut {
  std::vector<int> qidx;   // input query index of each pass query
};

// Plans, runs and collects one pass over queries [qa, qb).
constexpr kws_status PASS_TOO_WIDE = (kws_status)1;   // internal: retry with fewer queries

kws_status run_pass(kws_graph *g, const std::vector<QIn> &qs, int qa, int qb, int max_words, bool export_only,
                    uint8_t *export_dist, kws_result *out, FlatOut *flat) {
  Engine &E = g->eng;
  const kws_options &o = g->opt;
  const int32_t n = g->n;
  const int nq = qb - qa;
  Packing pk;
  pack(qs, qa, qb, o.share_lanes >= 0 && !export_only, pk);
  const int W = (int)pk.word_used.size();
  if (W > max_words) return PASS_TOO_WIDE;
  int T = 1;
  if (!export_only) {
    // pull gathers one 8T-byte piece per edge and tile (at least a 64-byte
    // line), the streaming kernels touch every padded word of every vertex
    double best = 0;
    for (int t = 1; t <= std::max(1, o.tile_words); t <<= 1) {
      const double tl = (W + t - 1) / t;
      const double cost = (double)g->m * tl * (4.0 + std::max(8.0 * t, 64.0)) +
                          (double)n * tl * t * 8.0 * 3.0 * 2.0;
      if (t == 1 || cost <= best) { best = cost; T = t; }
    }
  }
  const int tiles = (W + T - 1) / T, Wp = tiles * T;
  int D = 0;
  for (int q = qa; q < qb; q++) D = std::max(D, qs[q].dmax);
  int B = 0;
  while ((1 << B) <= D) B++;
  if (D == 0) B = 0;
  const int n_lanes = (int)pk.lanes.size();

  KWS_TRY(ensure_state(g, (size_t)n * Wp));
  KWS_TRY(E.flist.ensure(sizeof(int32_t) * (size_t)n, "frontier list"));
  KWS_TRY(E.flist_eoff.ensure(sizeof(int32_t) * (size_t)n, "frontier offsets"));

  // ---------------- plan buffer
  std::vector<int64_t> seed_off(n_lanes + 1, 0);
  std::vector<int32_t> seed_begin(n_lanes), lane_word(n_lanes), lane_bit(n_lanes);
  for (int l = 0; l < n_lanes; l++) {
    const LaneInfo &li = pk.lanes[l];
    const int32_t key = g->pre[li.kw];
    const int32_t b = g->h_inv_ptr[key], e = g->h_inv_ptr[key + g->span[li.kw]];
    seed_begin[l] = b;
    seed_off[l + 1] = seed_off[l] + (e - b);
    lane_word[l] = li.word;
    lane_bit[l] = li.bit;
  }
  std::vector<uint64_t> act((size_t)(D + 2) * Wp, 0);
  for (const LaneInfo &li : pk.lanes)
    for (int lv = 0; lv <= li.dmax; lv++) act[(size_t)lv * Wp + li.word] |= 1ull << li.bit;
  std::vector<int32_t> wq_ptr(Wp + 1, 0), wq(nq);
  for (int i = 0; i < nq; i++) wq_ptr[pk.q_word[i] + 1]++;
  for (int j = 0; j < Wp; j++) wq_ptr[j + 1] += wq_ptr[j];
  {
    std::vector<int32_t> fill(wq_ptr.begin(), wq_ptr.end() - 1);
    for (int i = 0; i < nq; i++) wq[fill[pk.q_word[i]]++] = i;
  }
  std::vector<int32_t> q_dmax(nq), q_nk(nq), q_kcap(nq), q_hoff(nq), q_coff(nq), q_ccap(nq), q_roff(nq + 1),
      q_kdoff(nq), q_eoff(nq), q_ecap(nq), q_boff(nq);
  std::vector<uint8_t> bits;
  std::vector<int32_t> qlanes;
  int64_t nhist = 0, ncand = 0, nslots = 0, nkd = 0, nedge = 0;
  for (int i = 0; i < nq; i++) {
    const QIn &Q = qs[qa + i];
    q_dmax[i] = Q.dmax;
    q_nk[i] = Q.nk;
    q_kcap[i] = std::min(Q.k, n);
    q_hoff[i] = (int32_t)nhist;
    nhist += Q.nk * Q.dmax + 1;
    q_ccap[i] = q_kcap[i] <= 2048 ? q_kcap[i] : pow2ceil(q_kcap[i]);
    q_coff[i] = (int32_t)ncand;
    ncand += q_ccap[i];
    q_roff[i] = (int32_t)nslots;
    nslots += q_kcap[i];
    q_kdoff[i] = (int32_t)nkd;
    nkd += (int64_t)q_kcap[i] * Q.nk;
    q_ecap[i] = Q.nk * Q.dmax;
    q_eoff[i] = (int32_t)nedge;
    nedge += (int64_t)q_kcap[i] * q_ecap[i];
    q_boff[i] = (int32_t)bits.size();
    bits.insert(bits.end(), pk.q_bits[i].begin(), pk.q_bits[i].begin() + Q.nk);
    qlanes.insert(qlanes.end(), pk.q_lanes[i].begin(), pk.q_lanes[i].begin() + Q.nk);
  }
  q_roff[nq] = (int32_t)nslots;
  if (nhist > INT32_MAX / 2 || ncand > INT32_MAX / 2 || nedge > INT32_MAX / 2 || nkd > INT32_MAX / 2)
    return fail(KWS_EOVERFLOW, "batch too large for one pass");
  int chunks = (int)std::min<int64_t>(512, std::max<int64_t>(1, ((int64_t)n + 2047) / 2048));
  int CH = (int)align_up((size_t)((n + chunks - 1) / chunks), 64);
  chunks = (n + CH - 1) / CH;
  const bool hist_lds = nhist <= 8192, te_lds = nq <= 2048;
  if ((size_t)chunks * (size_t)nhist > (size_t)INT32_MAX) return fail(KWS_EOVERFLOW, "histogram too large");

  Layout pl;
  const size_t o_act = pl.add(act.size() * 8), o_soff = pl.add(seed_off.size() * 8),
               o_sbeg = pl.add(seed_begin.size() * 4), o_lw = pl.add(lane_word.size() * 4),
               o_lb = pl.add(lane_bit.size() * 4), o_wqp = pl.add(wq_ptr.size() * 4), o_wq = pl.add(wq.size() * 4),
               o_qmask = pl.add((size_t)nq * 8), o_qword = pl.add((size_t)nq * 4), o_qdmax = pl.add((size_t)nq * 4),
               o_qnk = pl.add((size_t)nq * 4), o_qkcap = pl.add((size_t)nq * 4), o_qhoff = pl.add((size_t)nq * 4),
               o_qcoff = pl.add((size_t)nq * 4), o_qccap = pl.add((size_t)nq * 4),
               o_qroff = pl.add((size_t)(nq + 1) * 4), o_qkdoff = pl.add((size_t)nq * 4),
               o_qeoff = pl.add((size_t)nq * 4), o_qecap = pl.add((size_t)nq * 4), o_qboff = pl.add((size_t)nq * 4),
               o_bits = pl.add(bits.size() + 1), o_qlanes = pl.add(qlanes.size() * 4 + 4);
  KWS_TRY(E.h_plan.ensure(pl.size, "plan (host)"));
  KWS_TRY(E.plan.ensure(pl.size, "plan"));
  uint8_t *hp = E.h_plan.as<uint8_t>();
  auto put = [&](size_t off, const void *src, size_t bytes) { if (bytes) std::memcpy(hp + off, src, bytes); };
  put(o_act, act.data(), act.size() * 8);
  put(o_soff, seed_off.data(), seed_off.size() * 8);
  put(o_sbeg, seed_begin.data(), seed_begin.size() * 4);
  put(o_lw, lane_word.data(), lane_word.size() * 4);
  put(o_lb, lane_bit.data(), lane_bit.size() * 4);
  put(o_wqp, wq_ptr.data(), wq_ptr.size() * 4);
  put(o_wq, wq.data(), wq.size() * 4);
  put(o_qmask, pk.q_mask.data(), (size_t)nq * 8);
  put(o_qword, pk.q_word.data(), (size_t)nq * 4);
  put(o_qdmax, q_dmax.data(), (size_t)nq * 4);
  put(o_qnk, q_nk.data(), (size_t)nq * 4);
  put(o_qkcap, q_kcap.data(), (size_t)nq * 4);
  put(o_qhoff, q_hoff.data(), (size_t)nq * 4);
  put(o_qcoff, q_coff.data(), (size_t)nq * 4);
  put(o_qccap, q_ccap.data(), (size_t)nq * 4);
  put(o_qroff, q_roff.data(), (size_t)(nq + 1) * 4);
  put(o_qkdoff, q_kdoff.data(), (size_t)nq * 4);
  put(o_qeoff, q_eoff.data(), (size_t)nq * 4);
  put(o_qecap, q_ecap.data(), (size_t)nq * 4);
  put(o_qboff, q_boff.data(), (size_t)nq * 4);
  put(o_bits, bits.data(), bits.size());
  put(o_qlanes, qlanes.data(), qlanes.size() * 4);

  // ---------------- result arena (D2H) and zeroed scratch
  Layout al;
  const size_t a_stats = al.add((size_t)(D + 1) * 4 * 8), a_te = al.add((size_t)nq * 8),
               a_nroots = al.add((size_t)nq * 4), a_roots = al.add((size_t)nslots * 4),
               a_scores = al.add((size_t)nslots * 4), a_ecount = al.add((size_t)nslots * 4),
               a_kwdist = al.add((size_t)nkd), a_edges = al.add((size_t)nedge * 8);
  const size_t a_zero_end = a_nroots;   // stats and te are zeroed
  KWS_TRY(E.arena.ensure(al.size, "result arena"));
  KWS_TRY(E.h_arena.ensure(al.size, "result arena (host)"));
  Layout zl;
  const size_t z_live = zl.add((size_t)(D + 1) * Wp * 8), z_ccnt = zl.add((size_t)nq * 4),
               z_wcnt = zl.add(4), z_hist = zl.add((size_t)chunks * nhist * 4);
  KWS_TRY(E.zero_region.ensure(align_up(zl.size, 8), "counters"));
  KWS_TRY(E.work.ensure(sizeof(int4) * (size_t)std::max<int64_t>(nslots, 1), "select work"));
  KWS_TRY(E.cand.ensure(8 * (size_t)std::max<int64_t>(ncand, 1), "candidates"));
  KWS_TRY(E.qsel.ensure(sizeof(int32_t) * (size_t)nq * 4 + 16, "query selection"));

  KWS_HIP(hipMemcpyAsync(E.plan.p, hp, pl.size, hipMemcpyHostToDevice, g->stream));

  Pass P;
  std::memset(&P, 0, sizeof(P));
  P.n = n; P.tiles = tiles; P.Wp = Wp; P.G = std::min(64, pow2ceil(Wp)); P.D = D; P.B = B;
  P.nq = nq; P.n_lanes = n_lanes; P.chunks = chunks; P.CH = CH; P.nhist = (int32_t)nhist;
  P.hist_lds = hist_lds; P.te_lds = te_lds; P.force_dir = o.direction; P.alpha = o.alpha;
  P.total_seeds = seed_off[n_lanes]; P.n_hub = g->n_hub; P.total_slots = nslots; P.total_kd = nkd;
  for (int b = 0; b <= BIN_COUNT; b++) P.bin_begin[b] = g->bin_begin[b];
  P.pstride = (size_t)n * Wp;
  P.fwd_ptr = g->fwd_ptr; P.fwd_col = g->fwd_col; P.rev_ptr = g->rev_ptr; P.rev_col = g->rev_col;
  P.inv_vtx = g->inv_vtx; P.bin_vtx = g->bin_vtx; P.hub_v = g->hub_v; P.hub_b = g->hub_b; P.hub_e = g->hub_e;
  P.vis = E.vis.as<uint64_t>(); P.fr0 = E.fr0.as<uint64_t>(); P.fr1 = E.fr1.as<uint64_t>();
  P.nxt = E.nxt.as<uint64_t>(); P.planes = E.planes.as<uint64_t>();
  P.flist = E.flist.as<int32_t>(); P.flist_eoff = E.flist_eoff.as<int32_t>();
  uint8_t *dp = E.plan.as<uint8_t>();
  P.act = (const uint64_t *)(dp + o_act);
  P.lane_seed_off = (const int64_t *)(dp + o_soff);
  P.lane_seed_begin = (const int32_t *)(dp + o_sbeg);
  P.lane_word = (const int32_t *)(dp + o_lw);
  P.lane_bit = (const int32_t *)(dp + o_lb);
  P.word_q_ptr = (const int32_t *)(dp + o_wqp);
  P.word_q = (const int32_t *)(dp + o_wq);
  P.q_mask = (const uint64_t *)(dp + o_qmask);
  P.q_word = (const int32_t *)(dp + o_qword);
  P.q_dmax = (const int32_t *)(dp + o_qdmax);
  P.q_nk = (const int32_t *)(dp + o_qnk);
  P.q_kcap = (const int32_t *)(dp + o_qkcap);
  P.q_hoff = (const int32_t *)(dp + o_qhoff);
  P.q_coff = (const int32_t *)(dp + o_qcoff);
  P.q_ccap = (const int32_t *)(dp + o_qccap);
  P.q_roff = (const int32_t *)(dp + o_qroff);
  P.q_kdoff = (const int32_t *)(dp + o_qkdoff);
  P.q_eoff = (const int32_t *)(dp + o_qeoff);
  P.q_ecap = (const int32_t *)(dp + o_qecap);
  P.q_boff = (const int32_t *)(dp + o_qboff);
  P.bits = dp + o_bits;
  P.q_lane = (const int32_t *)(dp + o_qlanes);
  uint8_t *ar = E.arena.as<uint8_t>();
  uint8_t *zr = E.zero_region.as<uint8_t>();
  P.zero0 = (uint64_t *)ar; P.zero0_words = (int64_t)(a_zero_end / 8);
  P.zero1 = (uint64_t *)zr; P.zero1_words = (int64_t)(align_up(zl.size, 8) / 8);
  P.stats = (uint64_t *)(ar + a_stats);
  P.te = (uint64_t *)(ar + a_te);
  P.live = (uint64_t *)(zr + z_live);
  P.cand_cnt = (int32_t *)(zr + z_ccnt);
  P.work_cnt = (int32_t *)(zr + z_wcnt);
  P.hist = (int32_t *)(zr + z_hist);
  P.qsel = E.qsel.as<int32_t>();
  P.work = E.work.as<int4>();
  P.cand = E.cand.as<uint64_t>();
  P.r_nroots = (int32_t *)(ar + a_nroots);
  P.r_roots = (int32_t *)(ar + a_roots);
  P.r_scores = (int32_t *)(ar + a_scores);
  P.r_ecount = (int32_t *)(ar + a_ecount);
  P.r_kwdist = ar + a_kwdist;
  P.r_edges = (int2 *)(ar + a_edges);
  const int Wq = std::min(64, pow2ceil(Wp));

  if (export_only) {
    // seed + levels only, then export lane 0 of word 0
    DevBuf tmp;
    KWS_TRY(tmp.ensure((size_t)n, "distance export"));
    P.nq = nq;
    kws_status st = run_kernels(g, P, T, Wq);   // full pass keeps the code path identical
    if (st == KWS_OK) {
      k_export<1><<<clamp_grid(((int64_t)n + BLOCK - 1) / BLOCK), BLOCK, 0, g->stream>>>(P, tmp.as<uint8_t>());
      st = launch_check("export");
    }
    if (st == KWS_OK && hipMemcpyAsync(export_dist, tmp.p, (size_t)n, hipMemcpyDeviceToHost, g->stream) != hipSuccess)
      st = fail(KWS_EDEVICE, "export copy failed");
    if (st == KWS_OK && hipStreamSynchronize(g->stream) != hipSuccess) st = fail(KWS_EDEVICE, "export sync failed");
    tmp.release();
    return st;
  }

  if (o.use_graph > 0 && !g->prof.on) KWS_TRY(run_graph(g, P, T, Wq));
  else KWS_TRY(run_kernels(g, P, T, Wq));
  KWS_HIP(hipMemcpyAsync(E.h_arena.p, E.arena.p, al.size, hipMemcpyDeviceToHost, g->stream));
  KWS_HIP(hipStreamSynchronize(g->stream));
  KWS_TRY(g->prof.collect());

  // ---------------- unpack results
  const uint8_t *ha = E.h_arena.as<uint8_t>();
  const uint64_t *h_stats = (const uint64_t *)(ha + a_stats);
  const uint64_t *h_te = (const uint64_t *)(ha + a_te);
  const int32_t *h_nroots = (const int32_t *)(ha + a_nroots);
  const int32_t *h_roots = (const int32_t *)(ha + a_roots);
  const int32_t *h_scores = (const int32_t *)(ha + a_scores);
  const int32_t *h_ecount = (const int32_t *)(ha + a_ecount);
  const uint8_t *h_kwdist = ha + a_kwdist;
  const int2 *h_edges = (const int2 *)(ha + a_edges);
  for (int i = 0; i < nq; i++) {
    const QIn &Q = qs[qa + i];
    const int nr = h_nroots[i];
    if (flat) {
      FlatOut &F = *flat;
      F.kw.insert(F.kw.end(), Q.kw, Q.kw + Q.nk);
      F.kw_ptr.push_back((int64_t)F.kw.size());
      F.roots.insert(F.roots.end(), h_roots + q_roff[i], h_roots + q_roff[i] + nr);
      F.scores.insert(F.scores.end(), h_scores + q_roff[i], h_scores + q_roff[i] + nr);
      F.root_ptr.push_back((int64_t)F.roots.size());
      F.kw_dist.insert(F.kw_dist.end(), h_kwdist + q_kdoff[i], h_kwdist + q_kdoff[i] + (size_t)nr * Q.nk);
      F.dist_ptr.push_back((int64_t)F.kw_dist.size());
      for (int j = 0; j < nr; j++) {
        const int c = h_ecount[q_roff[i] + j];
        const int2 *src = h_edges + q_eoff[i] + (size_t)j * q_ecap[i];
        for (int t = 0; t < c; t++) { F.edge_src.push_back(src[t].x); F.edge_dst.push_back(src[t].y); }
        F.edge_ptr.push_back((int64_t)F.edge_src.size());
      }
      F.te.push_back((int64_t)h_te[i]);
      continue;
    }
    kws_result &r = out[qa + i];
    r.n_roots = nr;
    r.n_kw = Q.nk;
    r.te = (int64_t)h_te[i];
    r.kw = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max(1, Q.nk));
    r.roots = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max(1, nr));
    r.scores = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max(1, nr));
    r.kw_dist = (uint8_t *)malloc((size_t)std::max(1, nr * Q.nk));
    r.edge_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr + 1));
    int64_t ne = 0;
    for (int j = 0; j < nr; j++) ne += h_ecount[q_roff[i] + j];
    r.edge_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, ne));
    r.edge_dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, ne));
    if (!r.kw || !r.roots || !r.scores || !r.kw_dist || !r.edge_ptr || !r.edge_src || !r.edge_dst)
      return fail(KWS_ENOMEM, "host result allocation");
    std::memcpy(r.kw, Q.kw, sizeof(int32_t) * (size_t)Q.nk);
    if (nr) {
      std::memcpy(r.roots, h_roots + q_roff[i], sizeof(int32_t) * (size_t)nr);
      std::memcpy(r.scores, h_scores + q_roff[i], sizeof(int32_t) * (size_t)nr);
      std::memcpy(r.kw_dist, h_kwdist + q_kdoff[i], (size_t)nr * Q.nk);
    }
    r.edge_ptr[0] = 0;
    int64_t pos = 0;
    for (int j = 0; j < nr; j++) {
      const int c = h_ecount[q_roff[i] + j];
      const int2 *src = h_edges + q_eoff[i] + (size_t)j * q_ecap[i];
      for (int t = 0; t < c; t++) { r.edge_src[pos] = src[t].x; r.edge_dst[pos] = src[t].y; pos++; }
      r.edge_ptr[j + 1] = pos;
    }
  }
  // ---------------- pass statistics
  kws_batch_stats &bs = g->last;
  bs.queries += nq;
  bs.lanes += n_lanes;
  bs.lane_slots += pk.lane_slots;
  bs.words += W;
  bs.words_padded += Wp;
  bs.tiles += tiles;
  bs.tile_words = T;
  bs.levels = std::max(bs.levels, D);
  bs.passes += 1;
  for (int L = 0; L <= D && L <= KWS_MAX_DMAX; L++) {
    const uint64_t packed = h_stats[L * 4];
    const uint32_t nf = (uint32_t)(packed >> 32), mf = (uint32_t)packed;
    bs.frontier[L] += nf;
    bs.frontier_edges[L] += mf;
    bs.unfinished_edges[L] += (int64_t)h_stats[L * 4 + 1];
    if (L == D) break;
    int dir = 0;
    if (nf) dir = (o.direction == 1 || o.direction == 2) ? o.direction
                  : ((double)o.alpha * mf > (double)h_stats[L * 4 + 1] ? 2 : 1);
    bs.pulled[L] |= dir == 2;
  }
  return KWS_OK;
}

}  // namespace

void default_options(kws_options *o) {
  std::memset(o, 0, sizeof(*o));
  o->direction = 0;
  o->alpha = 8.0f;
  o->tile_words = 8;
  o->block = BLOCK;
  o->use_graph = 0;
  o->share_lanes = 1;
}

kws_status search(kws_graph *g, const kws_query *qs, int32_t nq, kws_result *out, FlatOut *flat) {
  if (!g || (!qs && nq > 0) || (!out && !flat && nq > 0) || nq < 0) return fail(KWS_EINVAL, "null argument");
  if (out)
    for (int i = 0; i < nq; i++) std::memset(&out[i], 0, sizeof(kws_result));
  std::vector<QIn> in(nq);
  for (int i = 0; i < nq; i++) {
    const kws_query &q = qs[i];
    if (q.n_kw < 1 || !q.kw) return fail(KWS_EINVAL, "query %d: needs at least one keyword", i);
    if (q.d_max < 0 || q.d_max > KWS_MAX_DMAX) return fail(KWS_EINVAL, "query %d: d_max %d outside 0..%d", i, q.d_max, KWS_MAX_DMAX);
    if (q.k < 0 || q.k > KWS_MAX_K) return fail(KWS_EINVAL, "query %d: k %d outside 0..%d", i, q.k, KWS_MAX_K);
    std::vector<int32_t> kw(q.kw, q.kw + q.n_kw);
    for (int32_t t : kw)
      if (t < 0 || t >= g->n_labels) return fail(KWS_EINVAL, "query %d: keyword %d out of range", i, t);
    std::sort(kw.begin(), kw.end());
    kw.erase(std::unique(kw.begin(), kw.end()), kw.end());
    if ((int)kw.size() > KWS_MAX_KW) return fail(KWS_EINVAL, "query %d: more than %d distinct keywords", i, KWS_MAX_KW);
    in[i].nk = (int32_t)kw.size();
    in[i].dmax = q.d_max;
    in[i].k = q.k;
    std::copy(kw.begin(), kw.end(), in[i].kw);
  }
  std::memset(&g->last, 0, sizeof(g->last));
  // split into passes that respect the word and memory limits
  const size_t per_word = (size_t)g->n * 8 * 8;   // vis, 2 frontiers, nxt, 4 planes
  size_t budget_words = g->mem_budget / std::max<size_t>(per_word, 1);
  const int max_words = (int)std::max<size_t>(1, std::min<size_t>(MAX_WORDS, budget_words));
  int qa = 0;
  while (qa < nq) {
    int qb = qa, used_words = 0, free_in_last = 0;
    while (qb < nq) {   // next-fit estimate of the words the queries need
      const int need = in[qb].nk;
      if (free_in_last >= need) { free_in_last -= need; qb++; continue; }
      if (used_words + 1 > max_words) break;
      used_words++;
      free_in_last = 64 - need;
      qb++;
    }
    if (qb == qa) return fail(KWS_ENOMEM, "device memory budget too small for one query");
    kws_status st;
    for (;;) {
      st = run_pass(g, in, qa, qb, max_words, false, nullptr, out, flat);
      if (st != PASS_TOO_WIDE) break;
      qb = qa + std::max(1, (qb - qa) * 7 / 8);
    }
    if (st != KWS_OK) {
      if (out)
        for (int i = 0; i < nq; i++) kws_result_free(&out[i]);
      g->eng.state_words = 0;   // force a clean reallocation (nxt must start at zero)
      return st;
    }
    qa = qb;
  }
  g->last.queries = nq;
  return KWS_OK;
}

kws_status debug_distances(kws_graph *g, int32_t kw, int32_t d_max, uint8_t *dist) {
  if (!g || !dist) return fail(KWS_EINVAL, "null argument");
  if (kw < 0 || kw >= g->n_labels) return fail(KWS_EINVAL, "keyword %d out of range", kw);
  if (d_max < 0 || d_max > KWS_MAX_DMAX) return fail(KWS_EINVAL, "d_max %d outside 0..%d", d_max, KWS_MAX_DMAX);
  std::vector<QIn> in(1);
  in[0].nk = 1; in[0].dmax = d_max; in[0].k = 0; in[0].kw[0] = kw;
  kws_status st = run_pass(g, in, 0, 1, 1, true, dist, nullptr, nullptr);
  if (st != KWS_OK) g->eng.state_words = 0;
  return st;
}

}  // namespace kws
