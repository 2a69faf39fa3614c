// Allocation-free distance export: the kernels of kws_debug_distances run
// on search state carved out of one fixed device array, so the call makes
// no device allocation of any kind (no hipMalloc or hipFree, no pinned host
// buffer, no library routine that allocates). For callers that cannot
// allocate: code under stream capture, tight serving loops, harnesses that
// forbid it.
//
// The array lives in this file as a static __device__ object, so every
// device the library runs on holds its own copy (allocated when the code
// object is loaded, held until the process ends). Host code never uses its
// name as an address: the device address is looked up once per device with
// hipGetSymbolAddress and kept. Calls are serialised process-wide (they all
// share each device's one array) and wait for their device work, so the
// next call never sees a half-written state; every region a call reads
// before writing is cleared by that call's own kernels.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "pass.h"

namespace kws {

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

std::mutex g_scratch_mu;                 // one call at a time: every call on a device shares its array
uint8_t *g_scratch_ptr[MAX_DEVICES] = {};

// The per-level tables of one lane, passed by value to the kernel that
// writes them into the array (no host-to-device copy from pageable memory).
struct LaneTablesArg {
  uint64_t act[KWS_MAX_DMAX + 2];        // level l: lanes allowed to reach distance l
  int8_t lvl[KWS_MAX_DMAX + 1];          // level l assigns distance l
  int64_t seed_off[2];                   // the lane's inverted-index slice [0, seeds)
  int32_t seed_begin, word, bit;
};

// Copies up to one blob of bytes, passed by value, into the array (the pass
// and step descriptors, which the kernels read from device memory).
struct Blob {
  uint8_t b[512];
};

__global__ void k_noalloc_put(const Blob blob, uint8_t *dst, int len) {
  for (int i = threadIdx.x; i < len; i += blockDim.x) dst[i] = blob.b[i];
}

kws_status put_bytes(uint8_t *dst, const void *src, size_t bytes, hipStream_t s) {
  const uint8_t *p = (const uint8_t *)src;
  for (size_t off = 0; off < bytes; off += sizeof(Blob)) {
    Blob b;
    const size_t len = std::min(sizeof(Blob), bytes - off);
    std::memcpy(b.b, p + off, len);
    k_noalloc_put<<<1, 256, 0, s>>>(b, dst + off, (int)len);
    KWS_HIP(hipGetLastError());
  }
  return KWS_OK;
}

__global__ void k_noalloc_tables(const LaneTablesArg t, int D, uint64_t *act, int8_t *lvl, int64_t *seed_off,
                                 int32_t *seed_begin, int32_t *lane_word, int32_t *lane_bit) {
  const int i = threadIdx.x;
  if (i < D + 2) act[i] = t.act[i];
  if (i < D + 1) lvl[i] = t.lvl[i];
  if (i < 2) seed_off[i] = t.seed_off[i];
  if (i == 0) { *seed_begin = t.seed_begin; *lane_word = t.word; *lane_bit = t.bit; }
}

// Bump layout of the array, every region 256-byte aligned.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return at;
  }
};

struct Regions {
  size_t vis, fr0, fr1, nxt, planes, flist, flist_eoff, flags, act, lvl, stats, live, seed_off, seed_begin,
      lane_word, lane_bit, pass, steps, end;
};

Regions layout(int32_t n, int D, int B) {
  Carve c;
  Regions r;
  const size_t words = (size_t)n;        // one word per vertex (a single lane)
  r.vis = c.take(8 * words);
  r.fr0 = c.take(8 * words);
  r.fr1 = c.take(8 * words);
  r.nxt = c.take(8 * words);
  r.planes = c.take(8 * words * (size_t)B);
  r.flist = c.take(4 * (size_t)n);
  r.flist_eoff = c.take(4 * (size_t)n);
  r.flags = c.take(2 * (size_t)n);
  r.act = c.take(8 * (size_t)(D + 2));
  r.lvl = c.take((size_t)(D + 1));
  r.stats = c.take(8 * (size_t)(D + 1) * STAT_WORDS);
  r.live = c.take(8 * (size_t)(D + 1));
  r.seed_off = c.take(16);
  r.seed_begin = c.take(4);
  r.lane_word = c.take(4);
  r.lane_bit = c.take(4);
  r.pass = c.take(sizeof(Pass));
  r.steps = c.take(sizeof(Step) * (size_t)(D + 1));
  r.end = c.off;
  return r;
}

// Device address of this device's array (looked up on the first call on
// the device, with that device current).
kws_status scratch_on(int dev, uint8_t **out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(KWS_EDEVICE, "device %d out of range", dev);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    KWS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(KWS_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = (uint8_t *)p;
  }
  *out = g_scratch_ptr[dev];
  return KWS_OK;
}

kws_status distances_noalloc(kws_graph *g, int32_t kw, int32_t d_max, uint8_t *dist_dev) {
  const int32_t n = g->n;
  const int D = d_max;
  int B = 0;
  while ((1 << B) <= D) B++;
  if (D == 0) B = 0;
  const Regions R = layout(n, D, B);
  if (R.end > SCRATCH_BYTES)
    return fail(KWS_ENOMEM,
                "the allocation-free path holds %zu bytes of search state per device; a graph of %d vertices "
                "at d_max %d needs %zu",
                SCRATCH_BYTES, n, d_max, R.end);
  int prev = 0;
  KWS_HIP(hipGetDevice(&prev));
  if (prev != g->device) KWS_HIP(hipSetDevice(g->device));
  struct Restore {
    int dev, prev;
    ~Restore() { if (dev != prev) (void)hipSetDevice(prev); }
  } restore{g->device, prev};
  uint8_t *base = nullptr;
  KWS_TRY(scratch_on(g->device, &base));
  hipStream_t s = g->stream;

  // the lane: keyword kw with radius d_max, bit 0 of word 0; its seeds are
  // the inverted-index slice of kw's type subtree
  LaneTablesArg t{};
  for (int lv = 0; lv <= D; lv++) t.act[lv] = 1ull;
  for (int lv = 0; lv <= D; lv++) t.lvl[lv] = (int8_t)lv;
  const int32_t key = g->pre[kw];
  const int32_t sb = g->h_inv_ptr[key], se = g->h_inv_ptr[key + g->span[kw]];
  t.seed_off[0] = 0;
  t.seed_off[1] = se - sb;
  t.seed_begin = sb;
  t.word = 0;
  t.bit = 0;
  k_noalloc_tables<<<1, 64, 0, s>>>(t, D, (uint64_t *)(base + R.act), (int8_t *)(base + R.lvl),
                                    (int64_t *)(base + R.seed_off), (int32_t *)(base + R.seed_begin),
                                    (int32_t *)(base + R.lane_word), (int32_t *)(base + R.lane_bit));
  KWS_HIP(hipGetLastError());

  Pass P;
  std::memset(&P, 0, sizeof(P));
  P.dev = (const Pass *)(base + R.pass);
  P.n = n;
  P.T = 1;
  P.tiles = 1;
  P.Wp = 1;
  P.W = 1;
  P.B = B;
  P.nq = 0;
  P.n_lanes = 1;
  P.force_dir = g->opt.direction;
  P.alpha = g->opt.alpha;
  P.count_te = 0;
  P.total_seeds = se - sb;
  P.n_hub = g->n_hub;
  for (int b = 0; b <= BIN_COUNT; b++) P.bin_begin[b] = g->bin_begin[b];
  P.pstride = (size_t)n;
  P.fwd_ptr = g->fwd_ptr; P.fwd_col = g->fwd_col; P.rev_ptr = g->rev_ptr; P.rev_col = g->rev_col;
  P.inv_vtx = g->inv_vtx; P.bin_vtx = g->bin_vtx; P.hub_v = g->hub_v; P.hub_b = g->hub_b; P.hub_e = g->hub_e;
  P.vis = (uint64_t *)(base + R.vis);
  P.fr0 = (uint64_t *)(base + R.fr0);
  P.fr1 = (uint64_t *)(base + R.fr1);
  P.nxt = (uint64_t *)(base + R.nxt);
  P.planes = (uint64_t *)(base + R.planes);
  P.flist = (int32_t *)(base + R.flist);
  P.flist_eoff = (int32_t *)(base + R.flist_eoff);
  P.lane_seed_off = (const int64_t *)(base + R.seed_off);
  P.lane_seed_begin = (const int32_t *)(base + R.seed_begin);
  P.lane_word = (const int32_t *)(base + R.lane_word);
  P.lane_bit = (const int32_t *)(base + R.lane_bit);
  P.seed_by_vertex = 0;
  P.seed_vb = BLOCK;
  // cleared by the seeding kernel before anything adds to them
  P.zero0 = (uint64_t *)(base + R.stats);
  P.zero0_words = (int64_t)(D + 1) * STAT_WORDS;
  P.zero1 = (uint64_t *)(base + R.live);
  P.zero1_words = D + 1;

  const uint64_t *act = (const uint64_t *)(base + R.act);
  const int8_t *lvl = (const int8_t *)(base + R.lvl);
  uint64_t *stats = (uint64_t *)(base + R.stats);
  uint64_t *live = (uint64_t *)(base + R.live);
  uint8_t *flags = base + R.flags;
  Step steps[KWS_MAX_DMAX + 1];
  for (int lv = -1; lv < D; lv++) {   // step lv expands level lv (none for lv = -1) into level lv + 1
    Step &S = steps[lv + 1];
    std::memset(&S, 0, sizeof(S));
    if (lv >= 0) {
      S.act_exp = act + (lv + 1);
      S.live_in = live + lv;
      S.st_in = stats + (size_t)lv * STAT_WORDS;
      S.fr_cur = (lv & 1) ? P.fr1 : P.fr0;
      S.flags_cur = flags + (size_t)(lv & 1) * n;
    }
    S.fr_next = ((lv + 1) & 1) ? P.fr1 : P.fr0;
    S.flags_next = flags + (size_t)((lv + 1) & 1) * n;
    S.act_new = act + (lv + 1);
    S.act_nn = act + (lv + 2);
    S.newlvl = lvl + (lv + 1);
    S.st_out = stats + (size_t)(lv + 1) * STAT_WORDS;
    S.live_out = live + (lv + 1);
    S.build_list = S.write_next = lv + 1 < D;
    S.dev = (const Step *)(base + R.steps) + (lv + 1);
  }
  KWS_TRY(put_bytes(base + R.pass, &P, sizeof(Pass), s));
  KWS_TRY(put_bytes(base + R.steps, steps, sizeof(Step) * (size_t)(D + 1), s));

  Profiler off;                        // no events: nothing is created or recorded
  KWS_TRY(launch_fill_zero(P.nxt, (size_t)n, s));   // the seeds are OR-ed into a cleared nxt
  KWS_TRY(launch_seed(P, s, off));
  KWS_TRY(launch_finalize(P, steps[0], s, off));
  for (int i = 1; i <= D; i++) {
    KWS_TRY(launch_expand(P, steps[i], s, off));
    KWS_TRY(launch_finalize(P, steps[i], s, off));
  }
  KWS_TRY(launch_export(P, dist_dev, s));
  KWS_HIP(hipStreamSynchronize(s));
  return KWS_OK;
}

}  // namespace

}  // namespace kws

kws_status kws_debug_distances_noalloc(kws_graph *g, int32_t kw, int32_t d_max, uint8_t *dist_dev) {
  kws::clear_error();
  if (!g || !dist_dev) return kws::fail(KWS_EINVAL, "null argument");
  if (kw < 0 || kw >= g->n_labels) return kws::fail(KWS_EINVAL, "keyword %d out of range", kw);
  if (d_max < 0 || d_max > KWS_MAX_DMAX) return kws::fail(KWS_EINVAL, "d_max %d outside 0..%d", d_max, KWS_MAX_DMAX);
  std::lock_guard<std::mutex> lk(g->mu);
  std::lock_guard<std::mutex> lk2(kws::g_scratch_mu);
  return kws::distances_noalloc(g, kw, d_max, dist_dev);
}
