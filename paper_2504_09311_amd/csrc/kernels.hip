// Device kernels of the keyword search and their launchers: seeding,
// level expansion by push (64-bit atomicOr into in-neighbours) or pull
// (each vertex missing lanes ORs its out-neighbours' frontier masks, no
// atomics, early exit), finalize with frontier compaction, root filter and
// score histogram, exact top-k with id-ordered ties, answer-graph walk.
//
// The push/pull choice is made on the device from the statistics the
// previous finalize wrote, so the launch sequence never depends on data.
#include <algorithm>
#include <cstring>

#include <map>
#include <mutex>

#include "pass.h"

namespace kws {

// Frontier statistics are spread over STAT_STRIPES cache lines (one stripe
// per group of blocks) so that no single address takes every block's atomic.
__device__ __forceinline__ uint64_t *stat_stripe(uint64_t *st, int64_t block) {
  return st + (size_t)(block % STAT_STRIPES) * STAT_STRIDE;
}

// Sums the stripes once per block (every thread of the block must call it)
// and returns 0 (nothing to expand), 1 (push) or 2 (pull).
__device__ int pick_dir(const uint64_t *st, float alpha, int force, uint32_t *nf_out = nullptr,
                        uint32_t *mf_out = nullptr) {
  __shared__ uint64_t s_tot[2];
  const int tid = threadIdx.x;
  uint64_t a = 0, b = 0;
  if (tid < STAT_STRIPES) { a = st[(size_t)tid * STAT_STRIDE]; b = st[(size_t)tid * STAT_STRIDE + 1]; }
  if (tid < 64)
    for (int off = 32; off > 0; off >>= 1) { a += __shfl_xor(a, off); b += __shfl_xor(b, off); }
  if (tid == 0) { s_tot[0] = a; s_tot[1] = b; }
  __syncthreads();
  const uint64_t packed = s_tot[0], mu = s_tot[1];
  __syncthreads();
  const uint32_t nf = (uint32_t)(packed >> 32), mf = (uint32_t)packed;
  if (nf_out) *nf_out = nf;
  if (mf_out) *mf_out = mf;
  if (nf == 0) return 0;                       // empty frontier: nothing to expand
  if (force == 1 || force == 2) return force;
  return (double)alpha * (double)mf > (double)mu ? 2 : 1;   // 1 push, 2 pull
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
__global__ __launch_bounds__(BLOCK) void k_seed(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
  const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, gsz = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = gid; i < P.zero0_words; i += gsz) P.zero0[i] = 0;
  for (int64_t i = gid; i < P.zero1_words; i += gsz) P.zero1[i] = 0;
  for (int64_t i = gid; i < P.zero2_words; i += gsz) P.zero2[i] = 0;
  __shared__ int s_lane;
  for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < P.total_seeds; base += gsz) {
    if (threadIdx.x == 0) {
      int lo = 0, hi = P.n_lanes;             // largest lane with lane_seed_off[lane] <= base
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (P.lane_seed_off[mid] <= base) lo = mid; else hi = mid;
      }
      s_lane = lo;
    }
    __syncthreads();
    int lo = s_lane;
    __syncthreads();
    const int64_t i = base + threadIdx.x;
    if (i >= P.total_seeds) continue;
    while (lo + 1 < P.n_lanes && P.lane_seed_off[lo + 1] <= i) lo++;
    const int32_t v = P.inv_vtx[P.lane_seed_begin[lo] + (int32_t)(i - P.lane_seed_off[lo])];
    const int word = P.lane_word[lo];
    const size_t idx = ((size_t)(word / T) * P.n + v) * T + (word % T);
    atomicOr((unsigned long long *)&P.nxt[idx], 1ull << P.lane_bit[lo]);
  }
}

// ---- seeding by vertex: the lanes a vertex starts are those whose keyword
// is one of its labels or (with a type hierarchy) an ancestor of one.
//
// type_walk: the threads of one row (SUB of them, this one `sub`) walk the
// type t and its ancestors, look each up in the pass's keyword hash and OR
// the lane masks of its entries into the LDS row (they split the entries).
__device__ __forceinline__ void type_walk(const Pass &P, int32_t t, uint64_t *row, int sub, int SUB) {
  const uint32_t hmask = (uint32_t)P.hcap - 1;
  for (; t >= 0; t = P.tparent ? P.tparent[t] : -1) {
    uint32_t h = ((uint32_t)t * 2654435761u) & hmask;
    int32_t key;
    while ((key = P.h_key[h]) != t && key != -1) h = (h + 1) & hmask;
    if (key != t) continue;
    const int32_t e0 = P.h_beg[h], e1 = e0 + P.h_cnt[h];
    for (int32_t e = e0 + sub; e < e1; e += SUB)
      atomicOr((unsigned long long *)&row[P.e_word[e]], (unsigned long long)P.e_mask[e]);
  }
}

// k_type_rows: with a type-row table, the walk runs once per type instead of
// once per (vertex, label): row t of the table ([n_types][Wp] words) holds
// the lanes type t starts, VB types per block round as in the seeding below.
__global__ __launch_bounds__(BLOCK) void k_type_rows(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
  extern __shared__ uint64_t s_rows[];   // [VB][Wp + 1]
  const int tid = threadIdx.x, VB = P.seed_vb, SUB = BLOCK / VB, RS = P.Wp + 1;
  const int vl = tid / SUB, sub = tid % SUB;
  for (int64_t t0 = (int64_t)blockIdx.x * VB; t0 < P.n_types; t0 += (int64_t)gridDim.x * VB) {
    for (int i = tid; i < VB * RS; i += BLOCK) s_rows[i] = 0;
    __syncthreads();
    if (t0 + vl < P.n_types) type_walk(P, (int32_t)(t0 + vl), s_rows + (size_t)vl * RS, sub, SUB);
    __syncthreads();
    const int nt = (int)min((int64_t)VB, (int64_t)P.n_types - t0);
    for (int i = tid; i < nt * P.Wp; i += BLOCK) {
      const int u = i / P.Wp, j = i - u * P.Wp;
      P.type_rows[(size_t)(t0 + u) * P.Wp + j] = s_rows[(size_t)u * RS + j];
    }
    __syncthreads();
  }
}

// seed_rows: the LDS rows of the VB vertices from v0 on, either from the
// type-row table (every (vertex, word) one thread, OR over the vertex's
// labels; a wavefront reads whole table rows) or by walking each label.
__device__ __forceinline__ void seed_rows(const Pass &P, int64_t v0, uint64_t *s_rows, int tid, int VB, int RS) {
  if (P.type_rows) {
    const int nv = (int)min((int64_t)VB, (int64_t)P.n - v0);
    for (int i = tid; i < nv * P.W; i += BLOCK) {
      const int u = i / P.W, j = i - u * P.W;
      const int32_t a = P.lab_ptr[v0 + u], b = P.lab_ptr[v0 + u + 1];
      uint64_t m = 0;
      for (int32_t l = a; l < b; l++) m |= P.type_rows[(size_t)P.lab[l] * P.Wp + j];
      s_rows[(size_t)u * RS + j] = m;
    }
    return;
  }
  const int SUB = BLOCK / VB, vl = tid / SUB, sub = tid % SUB;
  const int64_t v = v0 + vl;
  if (v < P.n) {
    const int32_t a = P.lab_ptr[v], b = P.lab_ptr[v + 1];
    for (int32_t i = a; i < b; i++) type_walk(P, P.lab[i], s_rows + (size_t)vl * RS, sub, SUB);
  }
}

// k_seed_vertex: a block takes VB vertices at a time and builds their rows of
// Wp words in LDS (seed_rows). The rows are then written to nxt tile by
// tile, so the stores follow the [tile][vertex][T] layout instead of
// scattering one word per (vertex, keyword).
template <int T>
__global__ __launch_bounds__(BLOCK) void k_seed_vertex(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
  extern __shared__ uint64_t s_rows[];   // [VB][Wp + 1] (one word of padding per row against bank conflicts)
  const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, gsz = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = gid; i < P.zero0_words; i += gsz) P.zero0[i] = 0;
  for (int64_t i = gid; i < P.zero1_words; i += gsz) P.zero1[i] = 0;
  for (int64_t i = gid; i < P.zero2_words; i += gsz) P.zero2[i] = 0;
  const int tid = threadIdx.x, VB = P.seed_vb, RS = P.Wp + 1;
  for (int64_t v0 = (int64_t)blockIdx.x * VB; v0 < P.n; v0 += (int64_t)gridDim.x * VB) {
    for (int i = tid; i < VB * RS; i += BLOCK) s_rows[i] = 0;
    __syncthreads();
    seed_rows(P, v0, s_rows, tid, VB, RS);
    __syncthreads();
    const int nv = (int)min((int64_t)VB, (int64_t)P.n - v0);
    for (int i = tid; i < P.tiles * VB * T; i += BLOCK) {
      const int tile = i / (VB * T), r = i % (VB * T), u = r / T, w = r % T;
      if (u >= nv) continue;
      const uint64_t m = s_rows[(size_t)u * RS + tile * T + w];
      if (m) P.nxt[((size_t)tile * P.n + v0 + u) * T + w] = m;
    }
    __syncthreads();
  }
}

// ---- the per-pass counters, zeroed before a seeding kernel that adds to
// some of them (k_seed_level0)
__global__ __launch_bounds__(BLOCK) void k_zero_pass(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
  const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, gsz = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = gid; i < P.zero0_words; i += gsz) P.zero0[i] = 0;
  for (int64_t i = gid; i < P.zero1_words; i += gsz) P.zero1[i] = 0;
  for (int64_t i = gid; i < P.zero2_words; i += gsz) P.zero2[i] = 0;
}

// ---- seeding by vertex fused with the finalize of level 0 (batched passes,
// where every word starts at level 0): the lookups of k_seed_vertex, then
// each vertex's row is its level-0 frontier, so it goes to vis and to the
// first frontier buffer directly (nxt is not touched), together with the
// frontier flag, the level-0 statistics and the live lanes that
// k_finalize would have produced from it.
template <int T>
__global__ __launch_bounds__(BLOCK) void k_seed_level0(const Pass *__restrict__ Pp, const Step *__restrict__ Sp) {
  const Pass &P = *Pp;
  const Step &S = *Sp;
  extern __shared__ uint64_t s_rows[];   // [VB][Wp + 1] rows, [Wp] live lanes, [VB] vertex flags
  const int tid = threadIdx.x, lane = tid & 63, VB = P.seed_vb, SUB = BLOCK / VB, RS = P.Wp + 1;
  uint64_t *s_live = s_rows + (size_t)VB * RS;
  uint32_t *s_vf = (uint32_t *)(s_live + P.Wp);
  const int vl = tid / SUB, sub = tid % SUB;
  uint64_t nf_acc = 0, mf_acc = 0, mu_acc = 0;
  for (int j = tid; j < P.Wp; j += BLOCK) s_live[j] = 0;
  for (int64_t v0 = (int64_t)blockIdx.x * VB; v0 < P.n; v0 += (int64_t)gridDim.x * VB) {
    for (int i = tid; i < VB * RS; i += BLOCK) s_rows[i] = 0;
    for (int i = tid; i < VB; i += BLOCK) s_vf[i] = 0;
    __syncthreads();
    seed_rows(P, v0, s_rows, tid, VB, RS);
    __syncthreads();
    const int64_t v = v0 + vl;
    const int nv = (int)min((int64_t)VB, (int64_t)P.n - v0);
    // per vertex: bit 0 any frontier lane, bit 1 a lane still to reach at level 1
    if (vl < nv) {
      const uint64_t *row = s_rows + (size_t)vl * RS;
      uint32_t fl = 0;
      for (int j = sub; j < P.W; j += SUB) {
        const uint64_t m = row[j];
        if (m) fl |= 1u;
        if (S.act_nn[j] & ~m) fl |= 2u;
      }
      if (fl) atomicOr(&s_vf[vl], fl);
    }
    for (int tile = 0; tile < P.tiles; tile++) {
      uint64_t lacc = 0;                  // every thread keeps one word (tid % T) of the tile
      for (int r = tid; r < VB * T; r += BLOCK) {
        const int u = r / T, w = r % T;
        if (u >= nv) break;
        const uint64_t m = s_rows[(size_t)u * RS + tile * T + w];
        const size_t idx = ((size_t)tile * P.n + v0 + u) * T + w;
        __builtin_nontemporal_store(m, &P.vis[idx]);
        if (S.write_next) __builtin_nontemporal_store(m, &S.fr_next[idx]);
        lacc |= m;
      }
      if (S.write_next) {
        for (int off = T; off < 64; off <<= 1) lacc |= __shfl_xor(lacc, off);
        if (lane < T && lacc) atomicOr((unsigned long long *)&s_live[tile * T + lane], lacc);
      }
    }
    __syncthreads();
    if (sub == 0 && vl < nv) {
      const uint32_t fl = s_vf[vl];
      if (S.build_list) S.flags_next[v] = (fl & 1u) ? 1 : 0;
      if (fl & 1u) { nf_acc++; mf_acc += (uint64_t)(P.rev_ptr[v + 1] - P.rev_ptr[v]); }
      if ((fl & 2u) && S.write_next) mu_acc += (uint64_t)(P.fwd_ptr[v + 1] - P.fwd_ptr[v]);
    }
    __syncthreads();
  }
  for (int off = 32; off > 0; off >>= 1) {
    nf_acc += __shfl_xor(nf_acc, off);
    mf_acc += __shfl_xor(mf_acc, off);
    mu_acc += __shfl_xor(mu_acc, off);
  }
  if (lane == 0) {
    uint64_t *st = stat_stripe(S.st_out, blockIdx.x);
    if (nf_acc) atomicAdd((unsigned long long *)&st[0], (unsigned long long)((nf_acc << 32) | mf_acc));
    if (mu_acc) atomicAdd((unsigned long long *)&st[1], (unsigned long long)mu_acc);
  }
  if (S.write_next) {
    __syncthreads();
    for (int j = tid; j < P.Wp; j += BLOCK)
      if (s_live[j]) atomicOr((unsigned long long *)&S.live_out[j], s_live[j]);
  }
}

// ---- k_seed_level0 from the type-row table, tiles of T >= 2 words: no LDS
// rows. A group of T / 2 threads owns one vertex, each thread two words of
// every tile (16-byte table loads, 16-byte stores of vis and the first
// frontier), so a wavefront writes the whole tile rows of 128 / T vertices
// in one contiguous run. The frontier flag, the level-0 statistics and the
// live lanes are reduced across the group and the wavefront by ballot and
// shuffles.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

template <int T>
__global__ __launch_bounds__(BLOCK) void k_seed_level0_tab(const Pass *__restrict__ Pp, const Step *__restrict__ Sp) {
  static_assert(T >= 2, "two words per thread");
  constexpr int G = T / 2, VPW = 64 / G;
  const Pass &P = *Pp;
  const Step &S = *Sp;
  extern __shared__ uint64_t s_live[];   // [Wp]
  const int tid = threadIdx.x, lane = tid & 63, t = lane % G;
  const uint64_t gmask = group_bits(lane, G);
  for (int j = tid; j < P.Wp; j += BLOCK) s_live[j] = 0;
  __syncthreads();
  uint64_t nf_acc = 0, mf_acc = 0, mu_acc = 0;
  const int64_t wave = ((int64_t)blockIdx.x * BLOCK + tid) / 64, nwaves = (int64_t)gridDim.x * (BLOCK / 64);
  for (int64_t v0 = wave * VPW; v0 < P.n; v0 += nwaves * VPW) {
    const int64_t v = v0 + lane / G;
    const bool valid = v < P.n;
    int32_t a = 0, b = 0;
    if (valid) { a = P.lab_ptr[v]; b = P.lab_ptr[v + 1]; }
    bool anyf = false, anyneed = false;
    for (int tile = 0; tile < P.tiles; tile++) {
      const int j = tile * T + 2 * t;
      u64x2 m = {0ull, 0ull};
      for (int32_t l = a; l < b; l++) m |= *(const u64x2 *)(P.type_rows + (size_t)P.lab[l] * P.Wp + j);
      if (valid) {
        const size_t idx = ((size_t)tile * P.n + v) * T + 2 * t;
        __builtin_nontemporal_store(m, (u64x2 *)(P.vis + idx));
        if (S.write_next) __builtin_nontemporal_store(m, (u64x2 *)(S.fr_next + idx));
        anyf |= (m.x | m.y) != 0;
        anyneed |= ((S.act_nn[j] & ~m.x) | (S.act_nn[j + 1] & ~m.y)) != 0;
      }
      if (S.write_next) {
        uint64_t lx = m.x, ly = m.y;
        for (int off = G; off < 64; off <<= 1) {
          lx |= __shfl_xor(lx, off);
          ly |= __shfl_xor(ly, off);
        }
        if (lane < G) {
          if (lx) atomicOr((unsigned long long *)&s_live[j], (unsigned long long)lx);
          if (ly) atomicOr((unsigned long long *)&s_live[j + 1], (unsigned long long)ly);
        }
      }
    }
    const bool fflag = (__ballot(anyf) & gmask) != 0, nflag = (__ballot(anyneed) & gmask) != 0;
    if (valid && t == 0) {
      if (S.build_list) S.flags_next[v] = fflag ? 1 : 0;
      if (fflag) { nf_acc++; mf_acc += (uint64_t)(P.rev_ptr[v + 1] - P.rev_ptr[v]); }
      if (nflag && S.write_next) mu_acc += (uint64_t)(P.fwd_ptr[v + 1] - P.fwd_ptr[v]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    nf_acc += __shfl_xor(nf_acc, off);
    mf_acc += __shfl_xor(mf_acc, off);
    mu_acc += __shfl_xor(mu_acc, off);
  }
  if (lane == 0) {
    uint64_t *st = stat_stripe(S.st_out, blockIdx.x);
    if (nf_acc) atomicAdd((unsigned long long *)&st[0], (unsigned long long)((nf_acc << 32) | mf_acc));
    if (mu_acc) atomicAdd((unsigned long long *)&st[1], (unsigned long long)mu_acc);
  }
  if (S.write_next) {
    __syncthreads();
    for (int j = tid; j < P.Wp; j += BLOCK)
      if (s_live[j]) atomicOr((unsigned long long *)&S.live_out[j], s_live[j]);
  }
}

// ---- finalize one step: new = nxt & ~vis & act_new; vis |= new; distance
// planes; next frontier buffer; nxt cleared; a frontier flag per vertex;
// the statistics that pick the direction of the next level (frontier size,
// its in-edges, out-edges of vertices still missing lanes), accumulated in
// registers and reduced once per wavefront. A pure streaming pass: the
// frontier list a push needs is built by k_compact, only for levels that push.
// T threads per vertex (one per word of a tile); each thread takes VU
// vertices per round and loads the words of up to 8 / VU tiles of each before
// any store, so every thread has up to 8 independent load pairs in flight
// (VU is 8 / min(tiles, 8), rounded to a power of two, and at most 4: with
// one tile, 4 vertices per thread leave room for more resident waves).
// Distance plane b (bit b of each lane's distance) is stored outright at the
// word's level 2^b, the first level that sets that bit: every lane not new
// there has a distance without bit b or none yet. Later levels with bit b
// OR their arrivals in. With S.clear_planes (words that may stop before
// level 2^b, as in the server) planes are cleared when the word starts and
// every level ORs.
template <int T, int VU>
__global__ __launch_bounds__(BLOCK) void k_finalize(const Pass *__restrict__ Pp, const Step *__restrict__ Sp) {
  const Pass &P = *Pp;
  const Step &S = *Sp;
  if (S.fused && pick_dir(S.st_in, P.alpha, P.force_dir) == 2) return;   // finalized by k_pull_fin
  extern __shared__ uint64_t s_live[];                    // [Wp]
  constexpr int G = T, VPB = BLOCK / T;
  constexpr int TG = 8 / VU;              // tiles per load group
  const int tid = threadIdx.x, gl = tid & (G - 1), lane = tid & 63;
  const uint64_t gmask = group_bits(lane, G);
  uint64_t *__restrict__ vis = P.vis;
  uint64_t *__restrict__ nxt = P.nxt;
  uint64_t *__restrict__ planes = P.planes;
  uint64_t *__restrict__ frn = S.fr_next;
  const size_t ps = P.pstride;
  for (int j = tid; j < P.Wp; j += BLOCK) s_live[j] = 0;
  __syncthreads();
  uint64_t live_acc[TG];                  // lanes with new frontier in the first TG tiles
#pragma unroll
  for (int k = 0; k < TG; k++) live_acc[k] = 0;
  uint64_t nf_acc = 0, mf_acc = 0, mu_acc = 0;
  for (int64_t vb = (int64_t)blockIdx.x * VPB * VU; vb < P.n; vb += (int64_t)gridDim.x * VPB * VU) {
    int64_t v[VU];
    uint64_t anyf[VU], anyneed[VU];
#pragma unroll
    for (int u = 0; u < VU; u++) { v[u] = vb + u * VPB + tid / G; anyf[u] = 0; anyneed[u] = 0; }
    for (int t0 = 0; t0 < P.tiles; t0 += TG) {
      uint64_t nxv[VU][TG], oldv[VU][TG];
#pragma unroll
      for (int u = 0; u < VU; u++)
#pragma unroll
        for (int k = 0; k < TG; k++) {
          const bool ok = v[u] < P.n && t0 + k < P.tiles;
          const size_t idx = ((size_t)(t0 + k) * P.n + v[u]) * T + gl;
          nxv[u][k] = ok ? __builtin_nontemporal_load(&nxt[idx]) : 0ull;
          oldv[u][k] = ok ? __builtin_nontemporal_load(&vis[idx]) : 0ull;
        }
#pragma unroll
      for (int k = 0; k < TG; k++) {
        if (t0 + k >= P.tiles) break;
        const int j = (t0 + k) * T + gl;
        const int nl = S.newlvl[j];
        const uint64_t an = S.act_new[j], ann = S.act_nn[j];
        // planes OR-ed into at this level: every bit of nl, except the bit
        // of a power-of-two level when planes are stored there outright
        const bool first_store = !S.clear_planes;
        const int rmw = first_store && (nl & (nl - 1)) == 0 ? 0 : nl;
        uint64_t lacc = 0;
#pragma unroll
        for (int u = 0; u < VU; u++) {
          if (v[u] >= P.n) continue;
          const size_t idx = ((size_t)(t0 + k) * P.n + v[u]) * T + gl;
          const uint64_t old = nl ? oldv[u][k] : 0ull;
          const uint64_t fnew = nxv[u][k] & ~old & an;
          const uint64_t nv = old | fnew;
          if (nl == 0) {
            vis[idx] = nv;
            if (S.clear_planes)
              for (int b = 0; b < P.B; b++) planes[b * ps + idx] = 0;
          } else {
            if (fnew) vis[idx] = nv;
            for (int b = 0; b < P.B; b++) {
              if (first_store && nl == (1 << b)) planes[b * ps + idx] = fnew;
              else if (fnew && ((rmw >> b) & 1)) planes[b * ps + idx] |= fnew;
            }
          }
          if (S.write_next) {
            if (!S.next_in_plane) __builtin_nontemporal_store(fnew, &frn[idx]);
            lacc |= fnew;
            anyneed[u] |= ann & ~nv;
          }
          if (nxv[u][k]) __builtin_nontemporal_store(0ull, &nxt[idx]);
          anyf[u] |= fnew;
        }
        if (t0 == 0) live_acc[k] |= lacc;
        else if (lacc) atomicOr((unsigned long long *)&s_live[j], lacc);
      }
    }
#pragma unroll
    for (int u = 0; u < VU; u++) {
      const bool fflag = (__ballot(anyf[u] != 0) & gmask) != 0;
      const bool nflag = (__ballot(anyneed[u] != 0) & gmask) != 0;
      if (v[u] < P.n && gl == 0) {
        if (S.build_list) S.flags_next[v[u]] = fflag ? 1 : 0;
        if (fflag) { nf_acc++; mf_acc += (uint64_t)(P.rev_ptr[v[u] + 1] - P.rev_ptr[v[u]]); }
        if (nflag) mu_acc += (uint64_t)(P.fwd_ptr[v[u] + 1] - P.fwd_ptr[v[u]]);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    nf_acc += __shfl_xor(nf_acc, off);
    mf_acc += __shfl_xor(mf_acc, off);
    mu_acc += __shfl_xor(mu_acc, off);
  }
  if (lane == 0) {
    uint64_t *st = stat_stripe(S.st_out, blockIdx.x);
    if (nf_acc) atomicAdd((unsigned long long *)&st[0], (unsigned long long)((nf_acc << 32) | mf_acc));
    if (mu_acc && S.write_next) atomicAdd((unsigned long long *)&st[1], (unsigned long long)mu_acc);
  }
  if (S.write_next) {
#pragma unroll
    for (int k = 0; k < TG; k++)   // OR over threads that own the same word, then one LDS atomic
      if (k < P.tiles) {
        uint64_t x = live_acc[k];
        for (int off = G; off < 64; off <<= 1) x |= __shfl_xor(x, off);
        if (lane < G && x) atomicOr((unsigned long long *)&s_live[k * T + gl], x);
      }
    __syncthreads();
    for (int j = tid; j < P.Wp; j += BLOCK)
      if (s_live[j]) atomicOr((unsigned long long *)&S.live_out[j], s_live[j]);
  }
}

// ---- compact: the frontier list (vertex, offset of its in-edges) from the
// frontier flags, for a level that expands by push. Wavefront ballot and
// prefix sums into LDS per chunk of CMP_CHUNK vertices; one global
// reservation per chunk.
constexpr int CMP_CHUNK = 2048;

__global__ __launch_bounds__(BLOCK) void k_compact(const Pass *__restrict__ Pp, const Step *__restrict__ Sp) {
  const Pass &P = *Pp;
  const Step &S = *Sp;
  if (pick_dir(S.st_in, P.alpha, P.force_dir) != 1) return;
  __shared__ int32_t s_lv[CMP_CHUNK], s_le[CMP_CHUNK];
  __shared__ unsigned long long s_acc, s_base;
  const int tid = threadIdx.x, lane = tid & 63;
  unsigned long long *cnt = (unsigned long long *)&S.st_in[2];   // list reservation counter (stripe 0)
  const int64_t nchunks = ((int64_t)P.n + CMP_CHUNK - 1) / CMP_CHUNK;
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    if (tid == 0) s_acc = 0;
    __syncthreads();
    const int64_t c0 = c * CMP_CHUNK, c1 = min((int64_t)P.n, c0 + CMP_CHUNK);
    for (int64_t vb = c0; vb < c1; vb += BLOCK) {
      const int64_t v = vb + tid;
      const bool take = v < c1 && S.flags_cur[v];
      const int32_t indeg = take ? P.rev_ptr[v + 1] - P.rev_ptr[v] : 0;
      const uint64_t bal = __ballot(take);
      const int32_t eincl = wave_incl_scan(indeg, lane);
      const int32_t wcnt = __popcll(bal), wedge = __shfl(eincl, 63);
      unsigned long long base = 0;
      if (lane == 0 && wcnt) base = atomicAdd(&s_acc, ((unsigned long long)wcnt << 32) | (uint32_t)wedge);
      base = __shfl(base, 0);
      if (take) {
        const int32_t pos = (int32_t)(base >> 32) + __popcll(bal & ((1ull << lane) - 1ull));
        s_lv[pos] = (int32_t)v;
        s_le[pos] = (int32_t)(uint32_t)base + eincl - indeg;
      }
    }
    __syncthreads();
    if (tid == 0) s_base = s_acc ? atomicAdd(cnt, s_acc) : 0ull;
    __syncthreads();
    const int32_t n_in = (int32_t)(s_acc >> 32);
    const int32_t bc = (int32_t)(s_base >> 32), be = (int32_t)(uint32_t)s_base;
    for (int i = tid; i < n_in; i += BLOCK) {
      P.flist[bc + i] = s_lv[i];
      P.flist_eoff[bc + i] = be + s_le[i];
    }
    __syncthreads();
  }
}

// ---- push: every frontier in-edge (p -> v) ORs v's frontier lanes into nxt[p]
// Wq threads per edge cover the words (power of two, <= 64).
template <int T>
__global__ __launch_bounds__(BLOCK) void k_push(const Pass *__restrict__ Pp, const Step *__restrict__ Sp, int Wq) {
  const Pass &P = *Pp;
  const Step &S = *Sp;
  uint32_t nf_u = 0, mf_u = 0;
  if (pick_dir(S.st_in, P.alpha, P.force_dir, &nf_u, &mf_u) != 1) return;
  const int32_t nf = (int32_t)nf_u;
  const int64_t mf = (int64_t)mf_u;
  const int EPB = BLOCK / Wq;
  const int tid = threadIdx.x, wq = tid & (Wq - 1), es = tid / Wq;
  const uint64_t *fr = S.fr_cur;
  const uint64_t *act = S.act_exp;
  const uint64_t *live = S.live_in;
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
    for (int word = wq; word < P.W; word += Wq) {
      const size_t tb = (size_t)(word / T) * P.n * T;
      const int w = word % T;
      uint64_t f = fr[tb + (size_t)v * T + w] & act[word] & live[word];
      if (!f) continue;
      f &= ~P.vis[tb + (size_t)p * T + w];
      if (f) atomicOr((unsigned long long *)&P.nxt[tb + (size_t)p * T + w], f);
    }
  }
}

// ---- the gather of one row by its group of S threads. Inside the gather a
// thread holds V adjacent words of the row (the pulls use V = 2 for 16-word
// tiles: 16-byte gathers, so one load instruction moves the rows of twice
// as many edges; 8-word tiles measured slower with it), LR = T / V threads
// cover a row and E = S / LR edge slots
// run side by side: thread (eo, w2) ORs words V*w2 .. V*w2 + V - 1 of the
// frontier rows of edges eo, eo + E, ... of [eb, ee), rounds of U edges
// per thread (the pulls use 4: the early-exit test comes after fewer
// gathers and the round holds fewer registers), and the group stops once
// it has every lane the vertex still misses. The column indices of a
// round are loaded coalesced, lane i of the group taking edge i
// (ceil(U / LR) loads of S indices), and each thread takes its U indices
// from those lanes by shuffle; the next round's loads are in flight while
// this round gathers. The caller loads the first round's indices
// (col_round at eb) into c, so that it can issue them ahead of the call.
// `need` comes and the result goes in the caller's layout, one word per
// thread (word gl % T); the result is already combined over the edge slots.
template <int LR, int U>
constexpr int col_loads() { return (U + LR - 1) / LR; }

template <int LR, int S, int U>
__device__ __forceinline__ void col_round(const int32_t *__restrict__ col, int32_t e0, int32_t ee, int gl,
                                          int32_t (&c)[col_loads<LR, U>()]) {
#pragma unroll
  for (int k = 0; k < col_loads<LR, U>(); k++) {
    const int32_t e = e0 + k * S + gl;
    c[k] = e < ee ? col[e] : -1;
  }
}

template <int T, int V, int S, int U>
__device__ __forceinline__ uint64_t gather_row(const uint64_t *__restrict__ fr, const int32_t *__restrict__ col,
                                               int32_t eb, int32_t ee, uint64_t need, int gl, uint64_t gmask,
                                               int32_t (&c)[col_loads<T / V, U>()]) {
  static_assert(V == 1 || (V == 2 && T >= 2), "one or two words per thread");
  constexpr int LR = T / V, E = S / LR, NL = col_loads<LR, U>();
  const int w = gl % T, w2 = gl % LR, eo = gl / LR;
  int32_t cn[NL], x[U];
  if (V == 1) {
    uint64_t acc = 0;
    for (int32_t e0 = eb; e0 < ee; e0 += E * U) {
#pragma unroll
      for (int u = 0; u < U; u++) x[u] = __shfl(c[u / LR], (u % LR) * E + eo, S);
#pragma unroll
      for (int k = 0; k < NL; k++) {
        const int32_t e = e0 + E * U + k * S + gl;
        cn[k] = e < ee ? col[e] : -1;
      }
      // a thread whose word has found every missing lane stops gathering
      const bool want = (acc & need) != need;
#pragma unroll
      for (int u = 0; u < U; u++)
        if (want && x[u] >= 0) acc |= fr[(size_t)x[u] * T + w];
      uint64_t r = acc;
#pragma unroll
      for (int off = LR; off < S; off <<= 1) r |= __shfl_xor(r, off);
      if ((__ballot((r & need) != need) & gmask) == 0) break;
#pragma unroll
      for (int k = 0; k < NL; k++) c[k] = cn[k];
    }
#pragma unroll
    for (int off = LR; off < S; off <<= 1) acc |= __shfl_xor(acc, off);
    return acc;
  } else {
    // this thread's two words' missing lanes, from the threads holding them
    const uint64_t nx = __shfl(need, 2 * w2, S), ny = __shfl(need, 2 * w2 + 1, S);
    uint64_t ax = 0, ay = 0;
    for (int32_t e0 = eb; e0 < ee; e0 += E * U) {
#pragma unroll
      for (int u = 0; u < U; u++) x[u] = __shfl(c[u / LR], (u % LR) * E + eo, S);
#pragma unroll
      for (int k = 0; k < NL; k++) {
        const int32_t e = e0 + E * U + k * S + gl;
        cn[k] = e < ee ? col[e] : -1;
      }
      const bool want = (ax & nx) != nx || (ay & ny) != ny;
#pragma unroll
      for (int u = 0; u < U; u++)
        if (want && x[u] >= 0) {
          const u64x2 f = *(const u64x2 *)(fr + (size_t)x[u] * T + 2 * w2);
          ax |= f.x;
          ay |= f.y;
        }
      uint64_t rx = ax, ry = ay;
#pragma unroll
      for (int off = LR; off < S; off <<= 1) {
        rx |= __shfl_xor(rx, off);
        ry |= __shfl_xor(ry, off);
      }
      if ((__ballot((rx & nx) != nx || (ry & ny) != ny) & gmask) == 0) break;
#pragma unroll
      for (int k = 0; k < NL; k++) c[k] = cn[k];
    }
#pragma unroll
    for (int off = LR; off < S; off <<= 1) {
      ax |= __shfl_xor(ax, off);
      ay |= __shfl_xor(ay, off);
    }
    // back to one word per thread: word w is component w % 2 of thread w / 2
    const uint64_t bx = __shfl(ax, w >> 1, S), by = __shfl(ay, w >> 1, S);
    return (w & 1) ? by : bx;
  }
}

// ---- pull: a group of S = T*E threads owns one row (or one hub chunk);
// thread (e, w) ORs word w of the frontier mask of every E-th out-neighbour.
// Early exit once the group has found every lane the vertex still misses.
// Rows are taken by the block in ranges [lo, hi) of the bin's (tile, row)
// items, item = tile * n_items + row.
template <int T, int S, bool SEG>
__device__ __forceinline__ void pull_rows(const Pass &P, const Step &SP, const int32_t *items, int64_t n_items,
                                          int tile, int bb, int bpt) {
  constexpr int GPB = BLOCK / S, U = 4, V = T == 16 ? 2 : 1;
  const int tid = threadIdx.x, gl = tid % S, w = gl % T, eo = gl / T, lane = tid & 63;
  const uint64_t gmask = group_bits(lane, S);
  const size_t tb = (size_t)tile * P.n * T;
  const uint64_t *fr = SP.fr_cur + tb;
  const uint64_t *vis = P.vis + tb;
  uint64_t *nxt = P.nxt + tb;
  const int word = tile * T + w;
  const uint64_t actw = SP.act_exp[word] & SP.live_in[word];
  const int32_t *col = P.fwd_col;
  // a row's descriptor (vertex, edge range, own vis word); the next row's
  // is loaded while this one gathers, so its chain of dependent loads
  // (bin entry, row bounds, vis) is not waited for between rows
  const int64_t stride = (int64_t)bpt * GPB;
  const auto load_row = [&](int64_t i, int32_t &rv, int32_t &rb, int32_t &re, uint64_t &ro) {
    if (i >= n_items) return;
    if (SEG) {
      rv = P.hub_v[i]; rb = P.hub_b[i]; re = P.hub_e[i];
    } else {
      rv = items[i]; rb = P.fwd_ptr[rv]; re = P.fwd_ptr[rv + 1];
    }
    ro = vis[(size_t)rv * T + w];
  };
  int64_t it = (int64_t)bb * GPB + tid / S;
  int32_t v = 0, eb = 0, ee = 0;
  uint64_t old = 0;
  load_row(it, v, eb, ee, old);
  int32_t c[col_loads<T / V, U>()];
  col_round<T / V, S, U>(col, eb, ee, gl, c);
  for (; it < n_items; it += stride) {
    int32_t vn = 0, ebn = 0, een = 0;
    uint64_t oldn = 0;
    load_row(it + stride, vn, ebn, een, oldn);
    const uint64_t need = actw & ~old;
    uint64_t acc = 0;
    const bool any = (__ballot(need != 0) & gmask) != 0;
    if (any) acc = gather_row<T, V, S, U>(fr, col, eb, ee, need, gl, gmask, c);
    // the next row's first column round, issued once its bounds are here
    col_round<T / V, S, U>(col, ebn, een, gl, c);
    if (any) {
      acc &= need;
      if (eo == 0 && acc) {
        if (SEG) atomicOr((unsigned long long *)&nxt[(size_t)v * T + w], acc);
        else nxt[(size_t)v * T + w] = acc;
      }
    }
    v = vn; eb = ebn; ee = een; old = oldn;
  }
}

// One launch covers every degree bin: blocks [boff[i], boff[i+1]) serve the
// i-th bin of PULL_ORDER, heaviest rows first (hub chunks, large, medium,
// small; inside a bin, rows by falling degree), so that the long rows start
// early instead of forming the tail. Inside a bin's range: tiles x
// blocks-per-tile, each block striding over the bin's rows.
struct PullGrid { int32_t boff[BIN_COUNT + 2]; };
constexpr int PULL_ORDER[BIN_COUNT + 1] = {BIN_COUNT, BIN_LARGE, BIN_MEDIUM, BIN_SMALL};

template <int T>
__global__ __launch_bounds__(BLOCK) void k_pull(const Pass *__restrict__ Pp, const Step *__restrict__ Sp, const PullGrid pg) {
  const Pass &P = *Pp;
  const Step &S = *Sp;
  if (pick_dir(S.st_in, P.alpha, P.force_dir) != 2) return;
  constexpr int S_SMALL = T, S_MED = (8 * T < 64 ? 8 * T : 64);
  const int bid = blockIdx.x;
  if (bid >= pg.boff[BIN_COUNT + 1]) return;   // the grid has one block even when every bin is empty
  int i = 0;
  while (i < BIN_COUNT && bid >= pg.boff[i + 1]) i++;
  const int b = PULL_ORDER[i];
  const int nblk = pg.boff[i + 1] - pg.boff[i];
  const int bpt = nblk / P.tiles, lb = bid - pg.boff[i];
  const int tile = lb / bpt, bb = lb % bpt;
  if (tile >= P.tiles) return;
  if (b == BIN_COUNT) {
    pull_rows<T, 64, true>(P, S, nullptr, P.n_hub, tile, bb, bpt);
    return;
  }
  const int32_t *items = P.bin_vtx + P.bin_begin[b];
  const int64_t n_items = P.bin_begin[b + 1] - P.bin_begin[b];
  if (b == BIN_SMALL) pull_rows<T, S_SMALL, false>(P, S, items, n_items, tile, bb, bpt);
  else if (b == BIN_MEDIUM) pull_rows<T, S_MED, false>(P, S, items, n_items, tile, bb, bpt);
  else pull_rows<T, 64, false>(P, S, items, n_items, tile, bb, bpt);
}

// ---- pull with the finalize fused in (pulled levels of batched passes,
// Step::fused). The grid is k_pull's: a group of S = T*E threads owns one
// (row, tile). After the gather, its lanes with eo == 0 hold the row's
// arrivals of their word and write what k_finalize would for that
// vertex-tile: vis where it gains lanes, the distance planes (stored
// outright at the plane's first level, OR-ed at later ones) and the next
// frontier (zero included). One writer per vertex-tile, so nothing is
// atomic and nxt is not touched. What needs every tile of a vertex (its
// frontier flag, the direction statistics) is left as one flag byte per
// vertex and tile (bit 0 new lanes, bit 1 lanes still to reach) for
// k_fin_stats. Hub rows (cut into chunks that merge with atomics into nxt)
// keep the unfused path and are finalized by k_fin_list; vertices without
// out-edges gain nothing and only get their zero next frontier, first-level
// planes and flag bytes.

// One vertex-word of a finalize at a level >= 1: writes vis, the planes
// and the next frontier; returns the new vis word. The active lanes of
// `gmask` hold the words of one vertex-tile row: where any of them gains
// lanes, all of them write vis (and the planes that are OR-ed at this
// level) back, so each row is one whole-line write instead of a partial
// line that the memory must read back to merge.
__device__ __forceinline__ uint64_t fin_word(const Pass &P, const Step &S, size_t idx, int j, uint64_t old,
                                             uint64_t fnew, uint64_t gmask) {
  const int nl = S.newlvl[j];
  const bool first_store = !S.clear_planes;
  const int rmw = first_store && (nl & (nl - 1)) == 0 ? 0 : nl;
  const uint64_t nv = old | fnew;
  const bool rowf = (__ballot(fnew != 0) & gmask) != 0;
  if (rowf) P.vis[idx] = nv;
  for (int b = 0; b < P.B; b++) {
    if (first_store && nl == (1 << b)) {
      P.planes[b * P.pstride + idx] = fnew;
    } else if (rowf && ((rmw >> b) & 1)) {
      uint64_t *pp = &P.planes[b * P.pstride + idx];
      *pp = *pp | fnew;
    }
  }
  if (S.write_next && !S.next_in_plane) __builtin_nontemporal_store(fnew, &S.fr_next[idx]);
  return nv;
}

template <int T, int S>
__device__ __forceinline__ void pull_fin_rows(const Pass &P, const Step &SP, const int32_t *items, int64_t n_items,
                                              int tile, int bb, int bpt, uint64_t &live_acc) {
  // rounds of 2 edges per thread when a thread gathers 16 bytes: in the
  // fused pull (state beyond the Infinity Cache) that measured faster than
  // 4; the unfused pull, run from cache-resident state, keeps 4
  constexpr int GPB = BLOCK / S, V = T == 16 ? 2 : 1, U = V == 2 ? 2 : 4;
  const int tid = threadIdx.x, gl = tid % S, w = gl % T, eo = gl / T, lane = tid & 63;
  const uint64_t gmask = group_bits(lane, S);
  const size_t tb = (size_t)tile * P.n * T;
  const uint64_t *fr = SP.fr_cur + tb;
  const int j = tile * T + w;
  const uint64_t actw = SP.act_exp[j] & SP.live_in[j];
  const uint64_t an = SP.act_new[j], ann = SP.act_nn[j];
  const int32_t *col = P.fwd_col;
  uint8_t *flags = SP.flags_tile + (size_t)tile * P.n;
  // the next row's descriptor is loaded while this row gathers (as in
  // pull_rows); the vis word read ahead is the next row's own, which no
  // other group writes
  const int64_t stride = (int64_t)bpt * GPB;
  const auto load_row = [&](int64_t i, int32_t &rv, int32_t &rb, int32_t &re, uint64_t &ro) {
    if (i >= n_items) return;
    rv = items[i]; rb = P.fwd_ptr[rv]; re = P.fwd_ptr[rv + 1];
    ro = P.vis[tb + (size_t)rv * T + w];
  };
  int64_t it = (int64_t)bb * GPB + tid / S;
  int32_t vc = 0, ebc = 0, eec = 0;
  uint64_t oldc = 0;
  load_row(it, vc, ebc, eec, oldc);
  int32_t c[col_loads<T / V, U>()];
  col_round<T / V, S, U>(col, ebc, eec, gl, c);
  for (; it < n_items; it += stride) {
    const int32_t v = vc, eb = ebc, ee = eec;
    const uint64_t old = oldc;
    load_row(it + stride, vc, ebc, eec, oldc);
    const size_t idx = tb + (size_t)v * T + w;
    const uint64_t need = actw & ~old;
    uint64_t acc = 0;
    if ((__ballot(need != 0) & gmask) != 0) acc = gather_row<T, V, S, U>(fr, col, eb, ee, need, gl, gmask, c);
    // the next row's first column round, issued once its bounds are here
    col_round<T / V, S, U>(col, ebc, eec, gl, c);
    bool anyf = false, anyneed = false;
    if (eo == 0) {
      const uint64_t fnew = acc & need & an;
      const uint64_t nv = fin_word(P, SP, idx, j, old, fnew, gmask);
      if (SP.write_next) live_acc |= fnew;
      anyf = fnew != 0;
      anyneed = (ann & ~nv) != 0;
    }
    const bool fflag = (__ballot(anyf) & gmask) != 0, nflag = (__ballot(anyneed) & gmask) != 0;
    if (gl == 0) flags[v] = (uint8_t)((fflag ? 1 : 0) | (nflag ? 2 : 0));
  }
}

// vertices without out-edges, one tile: nothing arrives; zero next frontier
// and first-level planes, zero flag byte (T threads per vertex)
template <int T>
__device__ __forceinline__ void fin_zero_rows(const Pass &P, const Step &SP, int tile, int bb, int bpt) {
  constexpr int GPB = BLOCK / T;
  const int tid = threadIdx.x, w = tid % T;
  const int j = tile * T + w;
  const int nl = SP.newlvl[j];
  const bool first_store = !SP.clear_planes;
  uint8_t *flags = SP.flags_tile + (size_t)tile * P.n;
  for (int64_t it = (int64_t)bb * GPB + tid / T; it < P.n_zero; it += (int64_t)bpt * GPB) {
    const int32_t v = P.zero_vtx[it];
    const size_t idx = (size_t)tile * P.n * T + (size_t)v * T + w;
    for (int b = 0; b < P.B; b++)
      if (first_store && nl == (1 << b)) P.planes[b * P.pstride + idx] = 0ull;
    if (SP.write_next && !SP.next_in_plane) __builtin_nontemporal_store(0ull, &SP.fr_next[idx]);
    if (w == 0) flags[v] = 0;
  }
}

// Live lanes of one word per thread: OR over the lanes that share the word
// (lane % T), one LDS atomic per word and wavefront, then one global atomic
// per word and block.
template <int T>
__device__ __forceinline__ void fin_live_out(const Step &S, uint64_t *s_live, int Wp, int j, uint64_t live_acc) {
  const int tid = threadIdx.x, lane = tid & 63;
  if (S.write_next) {
    uint64_t x = live_acc;
    for (int off = T; off < 64; off <<= 1) x |= __shfl_xor(x, off);
    if (lane < T && x) atomicOr((unsigned long long *)&s_live[j], x);
  }
  __syncthreads();
  if (S.write_next)
    for (int k = tid; k < Wp; k += BLOCK)
      if (s_live[k]) atomicOr((unsigned long long *)&S.live_out[k], s_live[k]);
}

// One launch, k_pull's grid plus the vertices without out-edges: blocks
// [boff[i], boff[i+1]) serve part i = hub chunks, large, medium, small
// rows, rows without out-edges; inside a part, tiles x blocks per tile.
struct FinGrid { int32_t boff[6]; };

template <int T>
__global__ __launch_bounds__(BLOCK) void k_pull_fin(const Pass *__restrict__ Pp, const Step *__restrict__ Sp, const FinGrid fg) {
  const Pass &P = *Pp;
  const Step &S = *Sp;
  if (pick_dir(S.st_in, P.alpha, P.force_dir) != 2) return;
  extern __shared__ uint64_t s_live[];   // [Wp]
  constexpr int S_SMALL = T, S_MED = (8 * T < 64 ? 8 * T : 64);
  for (int k = threadIdx.x; k < P.Wp; k += BLOCK) s_live[k] = 0;
  __syncthreads();
  const int bid = blockIdx.x;
  int part = 0;
  while (part < 5 && bid >= fg.boff[part + 1]) part++;
  uint64_t live_acc = 0;
  int tile = 0;
  if (part < 5) {
    const int nblk = fg.boff[part + 1] - fg.boff[part], lb = bid - fg.boff[part];
    const int bpt = nblk / P.tiles, bb = lb % bpt;
    tile = lb / bpt;
    if (tile < P.tiles) {
      if (part == 0) {
        pull_rows<T, 64, true>(P, S, nullptr, P.n_hub, tile, bb, bpt);
      } else if (part == 4) {
        fin_zero_rows<T>(P, S, tile, bb, bpt);
      } else {
        const int b = part == 1 ? BIN_LARGE : part == 2 ? BIN_MEDIUM : BIN_SMALL;
        const int32_t *items = P.bin_vtx + P.bin_begin[b];
        const int64_t n_items = P.bin_begin[b + 1] - P.bin_begin[b];
        if (b == BIN_SMALL) pull_fin_rows<T, S_SMALL>(P, S, items, n_items, tile, bb, bpt, live_acc);
        else if (b == BIN_MEDIUM) pull_fin_rows<T, S_MED>(P, S, items, n_items, tile, bb, bpt, live_acc);
        else pull_fin_rows<T, 64>(P, S, items, n_items, tile, bb, bpt, live_acc);
      }
    } else {
      tile = 0;
    }
  }
  fin_live_out<T>(S, s_live, P.Wp, tile * T + (int)(threadIdx.x % T), live_acc);
}

// The finalize of a list of vertices (the hub vertices of a fused pulled
// level): arrivals from nxt, which is cleared; T threads per vertex and
// tile; flag bytes as k_pull_fin writes them.
template <int T>
__global__ __launch_bounds__(BLOCK) void k_fin_list(const Pass *__restrict__ Pp, const Step *__restrict__ Sp, const int32_t *list, int64_t count) {
  const Pass &P = *Pp;
  const Step &S = *Sp;
  if (pick_dir(S.st_in, P.alpha, P.force_dir) != 2) return;
  extern __shared__ uint64_t s_live[];   // [Wp]
  constexpr int GPB = BLOCK / T;
  const int tid = threadIdx.x, w = tid % T, lane = tid & 63;
  const uint64_t gmask = group_bits(lane, T);
  for (int k = tid; k < P.Wp; k += BLOCK) s_live[k] = 0;
  __syncthreads();
  const int64_t items = count * P.tiles;
  for (int64_t it = (int64_t)blockIdx.x * GPB + tid / T; it < items; it += (int64_t)gridDim.x * GPB) {
    const int tile = (int)(it / count);
    const int32_t v = list[it % count];
    const int j = tile * T + w;
    const size_t idx = (size_t)tile * P.n * T + (size_t)v * T + w;
    const uint64_t old = P.vis[idx], nx = P.nxt[idx];
    const uint64_t fnew = nx & ~old & S.act_new[j];
    const uint64_t nv = fin_word(P, S, idx, j, old, fnew, gmask);
    if (nx) P.nxt[idx] = 0ull;
    if (fnew && S.write_next) atomicOr((unsigned long long *)&s_live[j], fnew);
    const bool fflag = (__ballot(fnew != 0) & gmask) != 0;
    const bool nflag = (__ballot((S.act_nn[j] & ~nv) != 0) & gmask) != 0;
    if (w == 0) S.flags_tile[(size_t)tile * P.n + v] = (uint8_t)((fflag ? 1 : 0) | (nflag ? 2 : 0));
  }
  __syncthreads();
  if (S.write_next)
    for (int k = tid; k < P.Wp; k += BLOCK)
      if (s_live[k]) atomicOr((unsigned long long *)&S.live_out[k], s_live[k]);
}

// Per vertex over its tiles' flag bytes: the frontier flag of the next
// level and the direction statistics (frontier vertices, their in-edges,
// out-edges of vertices still missing lanes), as k_finalize gives them.
__global__ __launch_bounds__(BLOCK) void k_fin_stats(const Pass *__restrict__ Pp, const Step *__restrict__ Sp) {
  const Pass &P = *Pp;
  const Step &S = *Sp;
  if (pick_dir(S.st_in, P.alpha, P.force_dir) != 2) return;
  const int lane = threadIdx.x & 63;
  uint64_t nf = 0, mf = 0, mu = 0;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < P.n; v += (int64_t)gridDim.x * BLOCK) {
    uint32_t f = 0;
    for (int t = 0; t < P.tiles; t++) f |= S.flags_tile[(size_t)t * P.n + v];
    if (S.build_list) S.flags_next[v] = (uint8_t)(f & 1u);
    if (f & 1u) { nf++; mf += (uint64_t)(P.rev_ptr[v + 1] - P.rev_ptr[v]); }
    if ((f & 2u) && S.write_next) mu += (uint64_t)(P.fwd_ptr[v + 1] - P.fwd_ptr[v]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    nf += __shfl_xor(nf, off);
    mf += __shfl_xor(mf, off);
    mu += __shfl_xor(mu, off);
  }
  if (lane == 0) {
    uint64_t *st = stat_stripe(S.st_out, blockIdx.x);
    if (nf) atomicAdd((unsigned long long *)&st[0], (unsigned long long)((nf << 32) | mf));
    if (mu) atomicAdd((unsigned long long *)&st[1], (unsigned long long)mu);
  }
}

// ---- score: per vertex and query, root test and score histogram per chunk;
// optionally the scanned-edge count te (in-degree of every vertex each lane
// expanded). A thread owns one vertex and holds the T words of one tile
// (vis and distance planes) in registers; a wavefront walks the words and
// their queries in lockstep, so the word -> query offsets and the query
// table (mask, histogram offset, query id, d_max, in word order) are read
// through the constant address space: scalar loads into SGPRs, operands of
// the vector ops without copies. With L the chunk's histogram (and the te
// sums) live in LDS and the histogram adds are LDS atomics; without L
// (batches too large for LDS) they go to global memory. TE (count_te) is a
// template argument so that the query loop carries no te work when it is
// off.
// With FIN the kernel also does the finalize of the last level (step F, in
// a batched pass, where nothing follows that level): it reads nxt beside
// vis and the planes, merges the arrivals in registers, writes back only
// what changed, clears nxt and adds the level's frontier statistics.
template <int T, bool L, bool TE, bool FIN, int PB>
__global__ __launch_bounds__(BLOCK) void k_score(const Pass *__restrict__ Pp, const Step *__restrict__ Fp) {
  const Pass &P = *Pp;
  extern __shared__ uint64_t s_dyn[];
  uint64_t *s_te = s_dyn;                                   // [nq] in word order (count_te)
  // the chunk histogram in LDS: two copies (a lane adds to the copy of its
  // parity, so lanes with equal scores meet half as often on one word), each
  // of hist_words words holding two 16-bit bins: bins below hist_split in
  // the low halves, the others (bin - hist_split) in the high halves; a
  // query's bins lie in one half. A bin counts at most the 128 lanes of one
  // parity in a block round, so a low half never carries into the high one
  uint32_t *s_hist = (uint32_t *)(s_dyn + (TE ? P.nq : 0));   // [2][hist_words]
  const int HW = P.hist_words, HS = P.hist_split;
  typedef const __attribute__((address_space(4))) QWord *QWordC;
  typedef const __attribute__((address_space(4))) int32_t *I32C;
  const QWordC qw = (QWordC)P.qw;
  const I32C wqp = (I32C)P.word_q_ptr;
  const int tid = threadIdx.x, lane = tid & 63;
  const int split = (P.CH + BLOCK - 1) / BLOCK;
  if (L && TE)
    for (int i = tid; i < P.nq; i += BLOCK) s_te[i] = 0;
  uint64_t nf_acc = 0, mf_acc = 0;        // FIN: frontier of the last level
  for (int64_t bid = blockIdx.x; bid < (int64_t)P.chunks * split; bid += gridDim.x) {
    const int c = (int)(bid / split), part = (int)(bid % split);
    if (L)
      for (int i = tid; i < 2 * HW; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    const int64_t cend = min((int64_t)P.n, (int64_t)(c + 1) * P.CH);
    const int64_t v = (int64_t)c * P.CH + (int64_t)part * BLOCK + tid;
    const bool valid = v < cend;
    const uint64_t indeg = (TE && valid) ? (uint64_t)(P.rev_ptr[v + 1] - P.rev_ptr[v]) : 0ull;
    // words held in registers at a time: at most 8 (a 16-word row in two
    // halves; whole rows need about 120 VGPRs, four waves per SIMD, and the
    // query loop wants the occupancy more than the row wants one read)
    constexpr int H = (T < 8 ? T : 8);
    bool anyf = false;
    for (int tile = 0; tile < P.tiles; tile++) {
#pragma unroll 1
      for (int h0 = 0; h0 < T; h0 += H) {
        if (wqp[tile * T + h0] == wqp[tile * T + h0 + H]) continue;   // no query in these words
        const size_t base = ((size_t)tile * P.n + (valid ? v : 0)) * T + h0;
        uint64_t vis[H], pl[PB][H];
#pragma unroll
        for (int w = 0; w < H; w++) vis[w] = 0ull;
#pragma unroll
        for (int b = 0; b < PB; b++)
#pragma unroll
          for (int w = 0; w < H; w++) pl[b][w] = 0ull;
        if (valid) {
          // 16-byte loads of the vertex's words (the tile row is 8T-byte aligned)
          if (H >= 2) {
#pragma unroll
            for (int w = 0; w < H; w += 2) {
              const ulonglong2 x = *(const ulonglong2 *)(P.vis + base + w);
              vis[w] = x.x; vis[w + 1 < H ? w + 1 : w] = H >= 2 ? x.y : x.x;
            }
#pragma unroll
            for (int b = 0; b < PB; b++)
              if (b < P.B)
#pragma unroll
                for (int w = 0; w < H; w += 2) {
                  const ulonglong2 x = *(const ulonglong2 *)(P.planes + b * P.pstride + base + w);
                  pl[b][w] = x.x; pl[b][w + 1 < H ? w + 1 : w] = x.y;
                }
          } else {
            vis[0] = P.vis[base];
#pragma unroll
            for (int b = 0; b < PB; b++)
              if (b < P.B) pl[b][0] = P.planes[b * P.pstride + base];
          }
          if (FIN) {
            // the last level's arrivals; words without a query have no lane
            // and so nothing in nxt. The row is updated in registers and
            // written back whole (16-byte stores) where it changed.
            bool rowf = false, rown = false;
            uint32_t store_pl = 0;                 // planes whose row is written
#pragma unroll
            for (int w = 0; w < H; w++) {
              const int j = tile * T + h0 + w;
              const int nl = Fp->newlvl[j];
              const uint64_t nx = __builtin_nontemporal_load(&P.nxt[base + w]);
              const uint64_t fnew = nx & ~vis[w] & Fp->act_new[j];
              rown |= nx != 0;
              if (fnew) {
                vis[w] |= fnew;
                rowf = true;
              }
#pragma unroll
              for (int b = 0; b < PB; b++)
                if (b < P.B) {
                  if (nl == (1 << b)) {                    // first level with bit b: stored outright
                    pl[b][w] = fnew;
                    store_pl |= 1u << b;
                  } else if (fnew && ((nl >> b) & 1)) {
                    pl[b][w] |= fnew;
                    store_pl |= 1u << b;
                  }
                }
            }
            if (rowf) anyf = true;
            if (H >= 2) {
#pragma unroll
              for (int w = 0; w < H; w += 2) {
                if (rowf) *(ulonglong2 *)(P.vis + base + w) = make_ulonglong2(vis[w], vis[w + 1 < H ? w + 1 : w]);
#pragma unroll
                for (int b = 0; b < PB; b++)
                  if ((store_pl >> b) & 1u)
                    *(ulonglong2 *)(P.planes + b * P.pstride + base + w) =
                        make_ulonglong2(pl[b][w], pl[b][w + 1 < H ? w + 1 : w]);
                if (rown) *(ulonglong2 *)(P.nxt + base + w) = make_ulonglong2(0ull, 0ull);
              }
            } else {
              if (rowf) P.vis[base] = vis[0];
#pragma unroll
              for (int b = 0; b < PB; b++)
                if ((store_pl >> b) & 1u) P.planes[b * P.pstride + base] = pl[b][0];
              if (rown) P.nxt[base] = 0ull;
            }
          }
#pragma unroll
          for (int w = 0; w < H; w++)
            if (tile * T + h0 + w >= P.W) {   // padding words carry no lane
              vis[w] = 0ull;
#pragma unroll
              for (int b = 0; b < PB; b++) pl[b][w] = 0ull;
            }
        }
#pragma unroll
        for (int w = 0; w < H; w++) {
          const int j = tile * T + h0 + w;
          // uniform by construction; readfirstlane lets the compiler see it
          // (the query index then stays scalar and the table loads are
          // scalar loads in every variant)
          const int qb = __builtin_amdgcn_readfirstlane(wqp[j]), qe = __builtin_amdgcn_readfirstlane(wqp[j + 1]);
          if (qb == qe || __ballot(vis[w] != 0) == 0) continue;
          // a plain loop over the word's queries; invalid lanes miss every
          // lane, so they are never roots. Planes past P.B hold zero in
          // registers and every d_max is below 2^P.B, so no plane needs a
          // bound check here.
          const uint64_t miss = valid ? ~vis[w] : ~0ull;
          // the next query's mask and histogram offset, loaded a query ahead
          // (the table ends with a zero entry, so no bound check)
          uint64_t m_next = qw[qb].mask;
          int32_t h_next = qw[qb].hoff;
#pragma unroll 2
          for (int qi = qb; qi < qe; qi++) {
            const uint64_t m = m_next;
            const int32_t hoff = h_next;
            m_next = qw[qi + 1].mask;
            h_next = qw[qi + 1].hoff;
            const bool root = (m & miss) == 0;
            if (TE) {
              const int q = qw[qi].q;
              const int dq = qw[qi].dmax;
              const uint64_t x = vis[w] & m;
              uint64_t eq = x;
#pragma unroll
              for (int b = 0; b < PB; b++) eq &= ((dq >> b) & 1) ? pl[b][w] : ~pl[b][w];
              uint64_t t = (uint64_t)(__popcll(x) - __popcll(eq)) * indeg;
              if (__ballot(t != 0)) {
                for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
                if (lane == 0) {
                  if (L) atomicAdd((unsigned long long *)&s_te[qi], (unsigned long long)t);
                  else atomicAdd((unsigned long long *)&P.te[q], (unsigned long long)t);
                }
              }
            }
            if (root) {                             // skipped as a whole when no lane has a root
              int sc = 0;
#pragma unroll
              for (int b = 0; b < PB; b++) sc += __popcll(pl[b][w] & m) << b;
              if (L) {
                const bool hi = hoff >= HS;      // per query: scalar
                atomicAdd(&s_hist[(lane & 1) * HW + (hi ? hoff - HS : hoff) + sc], hi ? 0x10000u : 1u);
              } else {
                atomicAdd(&P.hist[(size_t)c * P.nhist + hoff + sc], 1);
              }
            }
          }
        }
      }
    }
    if (FIN && anyf) { nf_acc++; mf_acc += (uint64_t)(P.rev_ptr[v + 1] - P.rev_ptr[v]); }
    __syncthreads();
    if (L)
      for (int i = tid; i < HW; i += BLOCK) {
        const uint32_t a = s_hist[i], b = s_hist[HW + i];
        const int32_t lo = (int32_t)((a & 0xFFFFu) + (b & 0xFFFFu)), hi = (int32_t)((a >> 16) + (b >> 16));
        if (lo && i < HS) atomicAdd(&P.hist[(size_t)c * P.nhist + i], lo);
        if (hi && HS + i < P.nhist) atomicAdd(&P.hist[(size_t)c * P.nhist + HS + i], hi);
      }
    __syncthreads();
  }
  if (L && TE) {
    __syncthreads();
    for (int i = tid; i < P.nq; i += BLOCK)
      if (s_te[i]) atomicAdd((unsigned long long *)&P.te[P.qw[i].q], (unsigned long long)s_te[i]);
  }
  if (FIN) {
    for (int off = 32; off > 0; off >>= 1) {
      nf_acc += __shfl_xor(nf_acc, off);
      mf_acc += __shfl_xor(mf_acc, off);
    }
    if (lane == 0 && nf_acc)
      atomicAdd((unsigned long long *)stat_stripe(Fp->st_out, blockIdx.x), (unsigned long long)((nf_acc << 32) | mf_acc));
  }
}

// ---- top-k early termination. After level L every lane's distances up to
// L are final, and a vertex that some keyword of a query has not reached
// will score at least L + 1 once it is a root. So a query with at least k
// complete roots (all its lanes reached) scoring at most L already has its
// top k, with every tie at L included: it stops expanding. Its lanes leave
// the activity table of the later levels unless a running query in the
// same word shares them; vis and the planes keep what level L left, which
// is exact for every vertex the score, the selection and the answer walk
// read. The distance planes whose first level is above L are not stored
// yet, and a distance of at most L has those bits clear, so they are not
// read here.
template <int T>
__global__ __launch_bounds__(BLOCK) void k_early_count(const Pass *__restrict__ Pp, int L) {
  const Pass &P = *Pp;
  extern __shared__ int32_t s_cnt[];   // [nq]
  const int tid = threadIdx.x, lane = tid & 63;
  for (int i = tid; i < P.nq; i += BLOCK) s_cnt[i] = 0;
  __syncthreads();
  int pv = 0;                            // planes stored by level L
  while (pv < P.B && (1 << pv) <= L) pv++;
  for (int64_t vb = (int64_t)blockIdx.x * BLOCK; vb < P.n; vb += (int64_t)gridDim.x * BLOCK) {
    const int64_t v = vb + tid;
    const bool valid = v < P.n;
    for (int j = 0; j < P.W; j++) {
      const int qb = P.word_q_ptr[j], qe = P.word_q_ptr[j + 1];
      if (qb == qe) continue;
      const size_t idx = ((size_t)(j / T) * P.n + (valid ? v : 0)) * T + (j % T);
      const uint64_t vis = valid ? P.vis[idx] : 0ull;
      if (__ballot(vis != 0) == 0) continue;
      uint64_t pl[4] = {0, 0, 0, 0};
      for (int b = 0; b < pv && b < 4; b++) pl[b] = valid ? P.planes[b * P.pstride + idx] : 0ull;
      for (int qi = qb; qi < qe; qi++) {
        const int q = P.word_q[qi];
        if (P.q_dmax[q] <= L || P.early_stop[q]) continue;
        const uint64_t m = P.q_mask[q];
        const bool root = valid && (m & ~vis) == 0;
        if (__ballot(root) == 0) continue;
        int sc = 0;
        for (int b = 0; b < pv && b < 4; b++) sc += __popcll(pl[b] & m) << b;
        const int c = __popcll(__ballot(root && sc <= L));
        if (lane == 0 && c) atomicAdd(&s_cnt[q], c);
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < P.nq; i += BLOCK)
    if (s_cnt[i]) atomicAdd(&P.early_cnt[i], s_cnt[i]);
}

__global__ __launch_bounds__(BLOCK) void k_early_apply(const Pass *__restrict__ Pp, int L) {
  const Pass &P = *Pp;
  const int tid = threadIdx.x;
  for (int q = tid; q < P.nq; q += BLOCK) {
    if (!P.early_stop[q] && P.q_dmax[q] > L && P.early_cnt[q] >= P.q_kcap[q]) P.early_stop[q] = L + 1;
    P.early_cnt[q] = 0;
  }
  __syncthreads();
  for (int j = tid; j < P.W; j += BLOCK) {
    uint64_t stop = 0, keep = 0;
    for (int qi = P.word_q_ptr[j]; qi < P.word_q_ptr[j + 1]; qi++) {
      const int q = P.word_q[qi];
      if (P.q_dmax[q] <= L) continue;    // its lanes are past their radius already
      if (P.early_stop[q]) stop |= P.q_mask[q];
      else keep |= P.q_mask[q];
    }
    const uint64_t clear = stop & ~keep;
    if (clear)
      for (int lv = L + 1; lv <= P.D + 1; lv++) P.act_tab[(size_t)lv * P.Wp + j] &= ~clear;
  }
}

// ---- threshold: per query, the score s* of the k-th root, how many ties at
// s* to take, and one work item per chunk that holds a selected root. A
// block of TH_BLOCK threads per query (a query's histograms span every
// chunk, and the ranks of ties run over the chunks in order).
constexpr int TH_BLOCK = 1024;

__device__ int32_t th_block_scan(int32_t x, int32_t *total) {
  __shared__ int32_t s_w[TH_BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int32_t incl = wave_incl_scan(x, lane);
  if (lane == 63) s_w[wid] = incl;
  __syncthreads();
  int32_t base = 0, all = 0;
  for (int w = 0; w < TH_BLOCK / 64; w++) {
    base += w < wid ? s_w[w] : 0;
    all += s_w[w];
  }
  __syncthreads();
  *total = all;
  return base + incl - x;
}

__global__ __launch_bounds__(TH_BLOCK) void k_threshold(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
  __shared__ int32_t tot[KWS_MAX_KW * KWS_MAX_DMAX + 1];
  __shared__ int32_t s_sel[4];
  const int tid = threadIdx.x;
  for (int q = blockIdx.x; q < P.nq; q += gridDim.x) {
    const int S1 = P.q_nk[q] * P.q_dmax[q] + 1, hoff = P.q_hoff[q];
    for (int s = tid; s < S1; s += TH_BLOCK) tot[s] = 0;
    __syncthreads();
    for (int64_t i = tid; i < (int64_t)P.chunks * S1; i += TH_BLOCK) {
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
      for (int base = 0; base < P.chunks; base += TH_BLOCK) {
        const int c = base + tid;
        int32_t t = 0, lt = 0;
        if (c < P.chunks) {
          const int32_t *h = P.hist + (size_t)c * P.nhist + hoff;
          t = h[sstar];
          for (int s = 0; s < sstar; s++) lt += h[s];
        }
        int32_t btot;
        const int32_t ex = th_block_scan(t, &btot) + carry;
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
// below s* and the first `need` ties overall (ranked across chunks). One
// wavefront per work item: ranks by ballot prefix counts (no block
// barriers), and the vis words of SU rounds of 64 vertices are loaded before
// any is used.
template <int T>
__global__ __launch_bounds__(BLOCK) void k_select(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
  constexpr int WAVES = BLOCK / 64, SU = 4;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  const int n_items = *P.work_cnt;
  for (int it = blockIdx.x * WAVES + wid; it < n_items; it += gridDim.x * WAVES) {
    const int4 wk = P.work[it];
    const int q = wk.x, c = wk.y, lt_c = wk.w;
    const int32_t sstar = P.qsel[q * 4 + 1], need = P.qsel[q * 4 + 2];
    const int word = P.q_word[q];
    const uint64_t m = P.q_mask[q];
    const size_t tb = (size_t)(word / T) * P.n * T;
    const int w = word % T;
    int32_t ties = wk.z, lts = 0;
    const int64_t v0 = (int64_t)c * P.CH, v1 = min((int64_t)P.n, v0 + P.CH);
    for (int64_t vb = v0; vb < v1 && !(lts >= lt_c && ties >= need); vb += 64 * SU) {
      uint64_t vw[SU];
#pragma unroll
      for (int u = 0; u < SU; u++) {
        const int64_t v = vb + u * 64 + lane;
        vw[u] = v < v1 ? P.vis[tb + (size_t)v * T + w] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < SU; u++) {
        const int64_t v = vb + u * 64 + lane;
        const bool root = v < v1 && (vw[u] & m) == m;
        int s = 0;
        if (root) {
          const size_t idx = tb + (size_t)v * T + w;
          for (int b = 0; b < P.B; b++) s += __popcll(P.planes[b * P.pstride + idx] & m) << b;
        }
        const bool lt = root && s < sstar, tie = root && s == sstar;
        const uint64_t tb_mask = __ballot(tie), lt_mask = __ballot(lt);
        const int32_t rank = ties + __popcll(tb_mask & below);
        if (lt || (tie && rank < need)) {
          const int32_t pos = atomicAdd(&P.cand_cnt[q], 1);
          P.cand[P.q_coff[q] + pos] = ((uint64_t)(uint32_t)s << 32) | (uint64_t)(uint32_t)v;
        }
        ties += __popcll(tb_mask);
        lts += __popcll(lt_mask);
      }
    }
  }
}

// ---- finish: order each query's candidates by (score, id); write roots,
// scores and the per-keyword distances.
template <int T>
__global__ __launch_bounds__(BLOCK) void k_finish(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
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

// ---- answer: one block per (query, root, keyword) walks from the root to
// the smallest-id out-neighbour one hop closer, writing the path into the
// keyword's segment of the root's edge slot; then one wave per (query, root)
// merges the segments: sort, drop repeats.
__device__ __forceinline__ int32_t block_min(int32_t v, int32_t *slot) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) atomicMin(slot, v);
  __syncthreads();
  const int32_t r = *slot;
  __syncthreads();
  return r;
}

// AB threads per walk scan AB neighbours per round: 512 when a pass has few
// walks (wider rounds end long rows sooner), 256 when it has many (more
// walks in flight).
template <int T, int AB>
__global__ __launch_bounds__(AB) void k_answer(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
  __shared__ int32_t s_best;
  constexpr int NSAMP = 4096;             // row samples held in LDS for the last hop
  __shared__ int32_t s_samp[NSAMP];
  const int tid = threadIdx.x;
  for (int64_t item = blockIdx.x; item < P.total_kd; item += gridDim.x) {
    int lo = 0, hi = P.nq;                      // query owning this (root, keyword) item
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (P.q_kdoff[mid] <= item) lo = mid; else hi = mid;
    }
    const int q = lo, nk = P.q_nk[q];
    const int rel = (int)(item - P.q_kdoff[q]), i = rel / nk, j = rel % nk;
    if (i >= P.qsel[q * 4 + 0]) continue;
    int d = P.r_kwdist[item];
    const int word = P.q_word[q], w = word % T, bit = P.bits[P.q_boff[q] + j];
    const size_t tb = (size_t)(word / T) * P.n * T;
    int2 *out = P.r_edges + P.q_eoff[q] + (size_t)i * P.q_ecap[q] + (size_t)j * P.q_dmax[q];
    const int32_t sb = P.qk_seed_b[P.q_boff[q] + j];
    const int64_t ns = P.qk_seed_e[P.q_boff[q] + j] - sb;
    int32_t x = P.r_roots[P.q_roff[q] + i];
    int h = 0;
    while (d > 0) {
      const int32_t e0 = P.fwd_ptr[x], e1 = P.fwd_ptr[x + 1];
      if (tid == 0) s_best = 0x7fffffff;
      __syncthreads();
      int32_t best = 0x7fffffff;
      if (d == 1 && ns * 4 < (int64_t)(e1 - e0)) {
        // last hop: the keyword's vertices are few compared with the row, so
        // look each of them up in the sorted row and keep the smallest hit:
        // first among NSAMP evenly spaced samples of the row held in LDS
        // (the whole row when it is that short), then within the one
        // segment between two samples
        const int32_t len = e1 - e0, step = (len + NSAMP - 1) / NSAMP, nsamp = (len + step - 1) / step;
        for (int k = tid; k < nsamp; k += AB) s_samp[k] = P.fwd_col[e0 + (int64_t)k * step];
        __syncthreads();
        int32_t mine = 0x7fffffff;
        for (int64_t k = tid; k < ns; k += AB) {
          const int32_t v = P.inv_vtx[sb + k];
          if (s_samp[0] > v) continue;
          int32_t lo = 0, hi = nsamp;        // last sample <= v
          while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (s_samp[mid] <= v) lo = mid; else hi = mid;
          }
          if (s_samp[lo] == v) { mine = min(mine, v); continue; }
          const int32_t seg_end = min(e1, e0 + lo * step + step);   // v lies after sample lo, before the next
          int32_t a = e0 + lo * step + 1, b = seg_end;
          while (a < b) {
            const int32_t mid = (a + b) >> 1;
            if (P.fwd_col[mid] < v) a = mid + 1; else b = mid;
          }
          if (a < seg_end && P.fwd_col[a] == v) mine = min(mine, v);
        }
        best = block_min(mine, &s_best);
      } else {
        // rows are sorted by neighbour id, so the qualifying neighbours of
        // the first round that has any include the smallest-id one. Most
        // walks stop in their first round, and every neighbour checked
        // costs up to three random loads, so the first round takes 64
        // neighbours (one wavefront) and the later ones AB
        for (int32_t eb = e0, rw = 64; eb < e1; eb += rw, rw = AB) {
          int32_t mine = 0x7fffffff;
          const int32_t e = eb + tid;
          const int32_t y = tid < rw && e < e1 ? P.fwd_col[e] : -1;
          if (y >= 0 && ((P.vis[tb + (size_t)y * T + w] >> bit) & 1ull) &&
              lane_dist(P, tb + (size_t)y * T + w, bit) == d - 1)
            mine = y;
          best = block_min(mine, &s_best);
          if (best != 0x7fffffff) break;
        }
      }
      if (best == 0x7fffffff || h >= P.q_dmax[q]) break;   // cannot happen for a BFS-consistent state
      if (tid == 0) out[h] = make_int2(x, best);
      h++;
      x = best;
      d--;
    }
  }
}

template <int T>
__global__ __launch_bounds__(BLOCK) void k_answer_merge(const Pass *__restrict__ Pp) {
  const Pass &P = *Pp;
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
__global__ __launch_bounds__(BLOCK) void k_export(const Pass *__restrict__ Pp, uint8_t *out) {
  const Pass &P = *Pp;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < P.n; v += (int64_t)gridDim.x * BLOCK) {
    const size_t idx = (size_t)v * T;
    out[v] = (P.vis[idx] & 1ull) ? (uint8_t)lane_dist(P, idx, 0) : (uint8_t)KWS_DIST_INF;
  }
}


// ============================================================ launchers

namespace {

inline unsigned clamp_grid(int64_t blocks) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 1 << 16));
}

// A per-batch size that sets a grid or an LDS size. In graph mode it is
// rounded up to a power of two, so batches of one shape launch identically
// and a captured graph replays for all of them (the kernels loop over
// their items, so a larger grid only adds blocks that find nothing to do).
inline int64_t launch_size(const Pass &P, int64_t x) {
  if (!P.graph_mode || x <= 1) return x;
  int64_t r = 1;
  while (r < x) r <<= 1;
  return r;
}

inline size_t score_lds(const Pass &P) {
  return P.hist_lds ? (size_t)launch_size(P, (int64_t)((P.count_te ? (size_t)P.nq * 8 : 0) +
                                                      8 * (size_t)P.hist_words))
                    : 0;
}

// Blocks of BLOCK threads that the whole device holds at once for this
// kernel and dynamic LDS size (occupancy x compute units), cached per kernel
// and LDS size.
int64_t resident_blocks(const void *fn, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<const void *, size_t>, int64_t> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({fn, lds});
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per_cu = 0;
  int64_t r = 1024;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BLOCK, lds) == hipSuccess && per_cu > 0 && cus > 0)
    r = (int64_t)per_cu * cus;
  cache[{fn, lds}] = r;
  return r;
}

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

__global__ void k_fill_u64(uint64_t *p, size_t count) {
  for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += (size_t)gridDim.x * BLOCK) p[i] = 0;
}

template <int T>
kws_status expand_t(const Pass &P, const Step &S, hipStream_t s, Profiler &prof) {
  const int Wq = std::min(64, P.Wp < 2 ? 1 : 1 << (32 - __builtin_clz((unsigned)P.Wp - 1)));
  {
    Timer t(prof, s, KC_PUSH);
    k_compact<<<clamp_grid(std::min<int64_t>(((int64_t)P.n + CMP_CHUNK - 1) / CMP_CHUNK, 4096)), BLOCK, 0, s>>>(P.dev, S.dev);
    k_push<T><<<2048, BLOCK, 0, s>>>(P.dev, S.dev, Wq);
  }
  KWS_TRY(launch_check("push"));
  constexpr int S_SMALL = T, S_MED = (8 * T < 64 ? 8 * T : 64);
  PullGrid pg;
  const int sizes[BIN_COUNT + 1] = {S_SMALL, S_MED, 64, 64};
  pg.boff[0] = 0;
  for (int i = 0; i <= BIN_COUNT; i++) {
    const int b = PULL_ORDER[i];
    const int64_t items = b < BIN_COUNT ? P.bin_begin[b + 1] - P.bin_begin[b] : P.n_hub;
    const int64_t gpb = BLOCK / sizes[b];
    const int64_t bpt = items ? std::min<int64_t>((items + gpb - 1) / gpb, 16384 / P.tiles + 1) : 0;
    pg.boff[i + 1] = pg.boff[i] + (int32_t)(bpt * P.tiles);
  }
  if (!S.fused) {
    Timer t(prof, s, KC_PULL);
    k_pull<T><<<(unsigned)std::max(1, pg.boff[BIN_COUNT + 1]), BLOCK, 0, s>>>(P.dev, S.dev, pg);
    return launch_check("pull");
  }
  // fused: k_pull's grid plus the vertices without out-edges (per tile);
  // then the hub vertices' finalize and the per-vertex flags and statistics
  FinGrid fg;
  for (int i = 0; i <= BIN_COUNT + 1; i++) fg.boff[i] = pg.boff[i];
  {
    const int64_t gpb = BLOCK / T, items = P.n_zero;
    const int64_t bpt = items ? std::min<int64_t>((items + gpb - 1) / gpb, 16384 / P.tiles + 1) : 0;
    fg.boff[BIN_COUNT + 2] = fg.boff[BIN_COUNT + 1] + (int32_t)(bpt * P.tiles);
  }
  const size_t lds = sizeof(uint64_t) * (size_t)P.Wp;
  {
    Timer t(prof, s, KC_PULL);
    k_pull_fin<T><<<(unsigned)std::max(1, fg.boff[BIN_COUNT + 2]), BLOCK, lds, s>>>(P.dev, S.dev, fg);
  }
  KWS_TRY(launch_check("pull"));
  {
    Timer t(prof, s, KC_FINALIZE);
    if (P.n_hubv > 0)
      k_fin_list<T><<<clamp_grid((P.n_hubv * P.tiles + BLOCK / T - 1) / (BLOCK / T)), BLOCK, lds, s>>>(P.dev, S.dev, P.hub_vtx, P.n_hubv);
    k_fin_stats<<<clamp_grid(std::min<int64_t>(((int64_t)P.n + BLOCK - 1) / BLOCK, 4096)), BLOCK, 0, s>>>(P.dev, S.dev);
  }
  return launch_check("fused finalize");
}

template <int T>
kws_status finalize_t(const Pass &P, const Step &S, hipStream_t s, Profiler &prof) {
  const int vu = P.tiles >= 8 ? 1 : P.tiles >= 4 ? 2 : 4;
  const int64_t per_block = (int64_t)(BLOCK / T) * vu;
  const size_t lds = sizeof(uint64_t) * (size_t)P.Wp;
  // one round of resident blocks that stride over the vertices: a second,
  // partial round of blocks would leave most of the chip idle at its end
  auto grid_for_kernel = [&](const void *fn) {
    const int64_t want = ((int64_t)P.n + per_block - 1) / per_block;
    return clamp_grid(std::min<int64_t>(want, resident_blocks(fn, lds)));
  };
  {
    Timer t(prof, s, KC_FINALIZE);
    switch (vu) {
      case 1: k_finalize<T, 1><<<grid_for_kernel((const void *)k_finalize<T, 1>), BLOCK, lds, s>>>(P.dev, S.dev); break;
      case 2: k_finalize<T, 2><<<grid_for_kernel((const void *)k_finalize<T, 2>), BLOCK, lds, s>>>(P.dev, S.dev); break;
      case 4: k_finalize<T, 4><<<grid_for_kernel((const void *)k_finalize<T, 4>), BLOCK, lds, s>>>(P.dev, S.dev); break;
      default: k_finalize<T, 8><<<grid_for_kernel((const void *)k_finalize<T, 8>), BLOCK, lds, s>>>(P.dev, S.dev); break;
    }
  }
  return launch_check("finalize");
}

// 16-word tiles with at most two planes hold whole rows (PB = 2); every
// other shape keeps room for four planes and rows of at most 8 words
template <int T, bool TE, bool FIN>
void score_launch(const Pass &P, const Step &F, int grid, size_t lds, hipStream_t s) {
  if constexpr (T == 16) {
    if (P.B <= 2) {
      if (P.hist_lds) k_score<T, true, TE, FIN, 2><<<grid, BLOCK, lds, s>>>(P.dev, F.dev);
      else k_score<T, false, TE, FIN, 2><<<grid, BLOCK, 0, s>>>(P.dev, F.dev);
      return;
    }
  }
  if (P.hist_lds) k_score<T, true, TE, FIN, 4><<<grid, BLOCK, lds, s>>>(P.dev, F.dev);
  else k_score<T, false, TE, FIN, 4><<<grid, BLOCK, 0, s>>>(P.dev, F.dev);
}

template <int T>
kws_status finish_t(const Pass &P, const Step *last, hipStream_t s, Profiler &prof) {
  if (P.nq == 0) {
    if (last) return launch_finalize(P, *last, s, prof);   // nothing to score: a plain finalize
    return KWS_OK;
  }
  {
    Timer t(prof, s, KC_SCORE);
    const int64_t split = (P.CH + BLOCK - 1) / BLOCK;
    const int grid = clamp_grid(launch_size(P, P.chunks * split));
    const size_t lds = score_lds(P);
    Step none;
    std::memset(&none, 0, sizeof(none));
    if (last) {
      if (P.count_te) score_launch<T, true, true>(P, *last, grid, lds, s);
      else score_launch<T, false, true>(P, *last, grid, lds, s);
    } else {
      if (P.count_te) score_launch<T, true, false>(P, none, grid, lds, s);
      else score_launch<T, false, false>(P, none, grid, lds, s);
    }
  }
  KWS_TRY(launch_check("score"));
  {
    Timer t(prof, s, KC_THRESHOLD);
    k_threshold<<<clamp_grid(launch_size(P, P.nq)), TH_BLOCK, 0, s>>>(P.dev);
  }
  KWS_TRY(launch_check("threshold"));
  {
    Timer t(prof, s, KC_SELECT);
    k_select<T><<<2048, BLOCK, 0, s>>>(P.dev);
  }
  KWS_TRY(launch_check("select"));
  {
    Timer t(prof, s, KC_FINISH);
    k_finish<T><<<clamp_grid(launch_size(P, P.nq)), BLOCK, 0, s>>>(P.dev);
  }
  KWS_TRY(launch_check("finish"));
  {
    Timer t(prof, s, KC_ANSWER);
    const int64_t waves = BLOCK / 64;
    const int64_t kd = launch_size(P, P.total_kd);
    if (kd <= 16384) k_answer<T, 512><<<clamp_grid(kd), 512, 0, s>>>(P.dev);
    else k_answer<T, 256><<<clamp_grid(kd), 256, 0, s>>>(P.dev);
    k_answer_merge<T><<<clamp_grid(launch_size(P, (P.total_slots + waves - 1) / waves)), BLOCK, 0, s>>>(P.dev);
  }
  return launch_check("answer");
}

#define KWS_DISPATCH_T(T_, CALL)                                   \
  switch (T_) {                                                     \
    case 1: { constexpr int TT = 1; return CALL; }                  \
    case 2: { constexpr int TT = 2; return CALL; }                  \
    case 4: { constexpr int TT = 4; return CALL; }                  \
    case 8: { constexpr int TT = 8; return CALL; }                  \
    case 16: { constexpr int TT = 16; return CALL; }                \
  }                                                                 \
  return fail(KWS_EINVAL, "tile width %d not supported", T_);

}  // namespace

// the type-row table of a pass, before its seeding kernel
void launch_type_rows(const Pass &P, hipStream_t s) {
  if (!P.type_rows || P.n_types <= 0) return;
  const int64_t blocks = (P.n_types + P.seed_vb - 1) / P.seed_vb;
  const size_t lds = sizeof(uint64_t) * (size_t)P.seed_vb * (size_t)(P.Wp + 1);
  k_type_rows<<<clamp_grid(std::min<int64_t>(blocks, 4096)), BLOCK, lds, s>>>(P.dev);
}

kws_status launch_seed(const Pass &P, hipStream_t s, Profiler &prof) {
  const int64_t zwords = launch_size(P, std::max(P.zero0_words, std::max(P.zero1_words, P.zero2_words)));
  const int64_t items = std::max<int64_t>(P.seed_by_vertex ? P.n : launch_size(P, P.total_seeds), zwords);
  if (P.seed_by_vertex) {
    Timer t(prof, s, KC_SEED);
    const int64_t vblocks = ((int64_t)P.n + P.seed_vb - 1) / P.seed_vb;
    const int64_t zblocks = (zwords + BLOCK - 1) / BLOCK;
    const int grid = clamp_grid(std::min<int64_t>(std::max<int64_t>(std::min<int64_t>(vblocks, 4096), zblocks), 65535));
    const size_t lds = sizeof(uint64_t) * (size_t)P.seed_vb * (size_t)(P.Wp + 1);
    launch_type_rows(P, s);
    switch (P.T) {
      case 1: k_seed_vertex<1><<<grid, BLOCK, lds, s>>>(P.dev); break;
      case 2: k_seed_vertex<2><<<grid, BLOCK, lds, s>>>(P.dev); break;
      case 4: k_seed_vertex<4><<<grid, BLOCK, lds, s>>>(P.dev); break;
      case 8: k_seed_vertex<8><<<grid, BLOCK, lds, s>>>(P.dev); break;
      case 16: k_seed_vertex<16><<<grid, BLOCK, lds, s>>>(P.dev); break;
      default: return fail(KWS_EINVAL, "tile width %d not supported", P.T);
    }
    return launch_check("seed");
  }
  {
    Timer t(prof, s, KC_SEED);
    switch (P.T) {
      case 1: k_seed<1><<<clamp_grid((items + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(P.dev); break;
      case 2: k_seed<2><<<clamp_grid((items + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(P.dev); break;
      case 4: k_seed<4><<<clamp_grid((items + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(P.dev); break;
      case 8: k_seed<8><<<clamp_grid((items + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(P.dev); break;
      case 16: k_seed<16><<<clamp_grid((items + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(P.dev); break;
      default: return fail(KWS_EINVAL, "tile width %d not supported", P.T);
    }
  }
  return launch_check("seed");
}

kws_status launch_seed_level0(const Pass &P, const Step &S, hipStream_t s, Profiler &prof) {
  Timer t(prof, s, KC_SEED);
  const int64_t zwords = launch_size(P, std::max(P.zero0_words, std::max(P.zero1_words, P.zero2_words)));
  if (zwords > 0) k_zero_pass<<<clamp_grid((zwords + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(P.dev);
  launch_type_rows(P, s);
  if (P.type_rows && P.T >= 2) {
    // T / 2 threads per vertex: 128 / T vertices per wavefront
    const int64_t per_block = (int64_t)(BLOCK / 64) * (128 / P.T);
    const int grid = clamp_grid(std::min<int64_t>(std::max<int64_t>(((int64_t)P.n + per_block - 1) / per_block, 1), 8192));
    const size_t lds_t = sizeof(uint64_t) * (size_t)P.Wp;
    switch (P.T) {
      case 2: k_seed_level0_tab<2><<<grid, BLOCK, lds_t, s>>>(P.dev, S.dev); break;
      case 4: k_seed_level0_tab<4><<<grid, BLOCK, lds_t, s>>>(P.dev, S.dev); break;
      case 8: k_seed_level0_tab<8><<<grid, BLOCK, lds_t, s>>>(P.dev, S.dev); break;
      case 16: k_seed_level0_tab<16><<<grid, BLOCK, lds_t, s>>>(P.dev, S.dev); break;
      default: return fail(KWS_EINVAL, "tile width %d not supported", P.T);
    }
    return launch_check("seed");
  }
  const int64_t vblocks = ((int64_t)P.n + P.seed_vb - 1) / P.seed_vb;
  const int grid = clamp_grid(std::min<int64_t>(std::max<int64_t>(vblocks, 1), 4096));
  const size_t lds = sizeof(uint64_t) * ((size_t)P.seed_vb * (size_t)(P.Wp + 1) + (size_t)P.Wp) +
                     sizeof(uint32_t) * (size_t)P.seed_vb;
  switch (P.T) {
    case 1: k_seed_level0<1><<<grid, BLOCK, lds, s>>>(P.dev, S.dev); break;
    case 2: k_seed_level0<2><<<grid, BLOCK, lds, s>>>(P.dev, S.dev); break;
    case 4: k_seed_level0<4><<<grid, BLOCK, lds, s>>>(P.dev, S.dev); break;
    case 8: k_seed_level0<8><<<grid, BLOCK, lds, s>>>(P.dev, S.dev); break;
    case 16: k_seed_level0<16><<<grid, BLOCK, lds, s>>>(P.dev, S.dev); break;
    default: return fail(KWS_EINVAL, "tile width %d not supported", P.T);
  }
  return launch_check("seed");
}

void graph_shape_key(const Pass &P, const std::vector<Step> &steps, bool fin_last, std::vector<int64_t> &key) {
  key.clear();
  // the descriptors' device addresses (the plan buffer of the I/O set) and
  // every value a launch above takes its grid, LDS size or variant from
  key.push_back((int64_t)(uintptr_t)P.dev);
  key.push_back(steps.empty() ? 0 : (int64_t)(uintptr_t)steps[0].dev);
  for (int64_t x : {(int64_t)P.T, (int64_t)P.tiles, (int64_t)P.Wp, (int64_t)P.B, (int64_t)P.n,
                    (int64_t)P.seed_by_vertex, (int64_t)P.seed_vb, (int64_t)P.hist_lds, (int64_t)P.count_te,
                    (int64_t)(P.type_rows != nullptr), P.n_types,
                    (int64_t)fin_last, (int64_t)steps.size(), (int64_t)(P.nq == 0)})
    key.push_back(x);
  const int64_t split = (P.CH + BLOCK - 1) / BLOCK, waves = BLOCK / 64;
  for (int64_t x : {std::max(P.zero0_words, std::max(P.zero1_words, P.zero2_words)), P.total_seeds,
                    P.chunks * split, (int64_t)P.nq, P.total_kd, (P.total_slots + waves - 1) / waves})
    key.push_back(launch_size(P, x));
  key.push_back((int64_t)score_lds(P));
  key.push_back((int64_t)P.early);
  for (const Step &S : steps) key.push_back((int64_t)S.fused);
}

kws_status launch_expand(const Pass &P, const Step &S, hipStream_t s, Profiler &prof) {
  KWS_DISPATCH_T(P.T, expand_t<TT>(P, S, s, prof))
}

kws_status launch_finalize(const Pass &P, const Step &S, hipStream_t s, Profiler &prof) {
  KWS_DISPATCH_T(P.T, finalize_t<TT>(P, S, s, prof))
}

kws_status launch_finish(const Pass &P, hipStream_t s, Profiler &prof, const Step *last) {
  KWS_DISPATCH_T(P.T, finish_t<TT>(P, last, s, prof))
}

kws_status launch_early(const Pass &P, int L, hipStream_t s, Profiler &prof) {
  if (!P.early || P.nq == 0) return KWS_OK;
  Timer t(prof, s, KC_EARLY);
  const int grid = clamp_grid(std::min<int64_t>(((int64_t)P.n + BLOCK - 1) / BLOCK, 4096));
  const size_t lds = sizeof(int32_t) * (size_t)launch_size(P, P.nq);   // a replay may carry more queries
  switch (P.T) {
    case 1: k_early_count<1><<<grid, BLOCK, lds, s>>>(P.dev, L); break;
    case 2: k_early_count<2><<<grid, BLOCK, lds, s>>>(P.dev, L); break;
    case 4: k_early_count<4><<<grid, BLOCK, lds, s>>>(P.dev, L); break;
    case 8: k_early_count<8><<<grid, BLOCK, lds, s>>>(P.dev, L); break;
    case 16: k_early_count<16><<<grid, BLOCK, lds, s>>>(P.dev, L); break;
    default: return fail(KWS_EINVAL, "tile width %d not supported", P.T);
  }
  KWS_TRY(launch_check("early count"));
  k_early_apply<<<1, BLOCK, 0, s>>>(P.dev, L);
  return launch_check("early apply");
}

kws_status launch_export(const Pass &P, uint8_t *out, hipStream_t s) {
  if (P.T != 1) return fail(KWS_EINVAL, "distance export needs a one-word pass");
  k_export<1><<<clamp_grid(((int64_t)P.n + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(P.dev, out);
  return launch_check("export");
}

kws_status launch_fill_zero(uint64_t *p, size_t words, hipStream_t s) {
  if (words == 0) return KWS_OK;
  k_fill_u64<<<clamp_grid((int64_t)((words + BLOCK - 1) / BLOCK)), BLOCK, 0, s>>>(p, words);
  return launch_check("fill");
}

}  // namespace kws
