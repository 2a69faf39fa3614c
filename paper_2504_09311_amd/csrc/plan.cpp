// Host-side planning shared by the batched path and the server.
#include <algorithm>
#include <cstring>
#include <unordered_map>

#include "engine.h"

namespace kws {

namespace {
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int pow2ceil(int x) { int p = 1; while (p < x) p <<= 1; return p; }

struct Layout {
  size_t size = 0;
  size_t add(size_t bytes, size_t align = 256) {
    size = align_up(size, align);
    const size_t off = size;
    size += bytes;
    return off;
  }
};
}  // namespace

kws_status normalize_query(const kws_graph *g, const kws_query &q, int i, QIn &out) {
  if (q.n_kw < 1 || !q.kw) return fail(KWS_EINVAL, "query %d: needs at least one keyword", i);
  if (q.d_max < 0 || q.d_max > KWS_MAX_DMAX)
    return fail(KWS_EINVAL, "query %d: d_max %d outside 0..%d", i, q.d_max, KWS_MAX_DMAX);
  if (q.k < 0 || q.k > KWS_MAX_K) return fail(KWS_EINVAL, "query %d: k %d outside 0..%d", i, q.k, KWS_MAX_K);
  std::vector<int32_t> kw(q.kw, q.kw + q.n_kw);
  for (int32_t t : kw)
    if (t < 0 || t >= g->n_labels) return fail(KWS_EINVAL, "query %d: keyword %d out of range", i, t);
  std::sort(kw.begin(), kw.end());
  kw.erase(std::unique(kw.begin(), kw.end()), kw.end());
  if ((int)kw.size() > KWS_MAX_KW) return fail(KWS_EINVAL, "query %d: more than %d distinct keywords", i, KWS_MAX_KW);
  out.nk = (int32_t)kw.size();
  out.dmax = q.d_max;
  out.k = q.k;
  std::copy(kw.begin(), kw.end(), out.kw);
  return KWS_OK;
}

// A query needs nk lanes in one word. With sharing, a keyword already in
// that word with the same d_max is reused; among words with room the one
// that shares most wins (first on ties); otherwise a new word is opened.
void pack_queries(const std::vector<QIn> &qs, int qa, int qb, bool share, Packing &pk) {
  pk = Packing();
  std::unordered_map<uint64_t, std::vector<std::array<int32_t, 2>>> where;   // (kw, d) -> (word, bit)
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
    Placed pl;
    pl.word = best;
    for (int j = 0; j < Q.nk; j++) {
      const uint64_t key = ((uint64_t)(uint32_t)Q.kw[j] << 8) | (uint64_t)Q.dmax;
      int bit = -1;
      if (share) {
        auto it = where.find(key);
        if (it != where.end())
          for (auto &wb : it->second)
            if (wb[0] == best) { bit = wb[1]; break; }
      }
      if (bit < 0) {
        bit = pk.word_used[best]++;
        pk.lanes.push_back({Q.kw[j], Q.dmax, best, bit});
        where[key].push_back({best, bit});
      }
      pl.bits[j] = (uint8_t)bit;
      pl.mask |= 1ull << bit;
    }
    pk.placed.push_back(pl);
    pk.lane_slots += Q.nk;
  }
}

void LaneTables::add(const kws_graph *g, const LaneInfo &li) {
  const int32_t key = g->pre[li.kw];
  const int32_t b = g->h_inv_ptr[key], e = g->h_inv_ptr[key + g->span[li.kw]];
  seed_begin.push_back(b);
  seed_off.push_back(seed_off.back() + (e - b));
  word.push_back(li.word);
  bit.push_back(li.bit);
  kw.push_back(li.kw);
}

// Open-addressing table keyword -> entries [(word, lane mask)], one entry
// per word that holds lanes of the keyword; probing is linear from
// (kw * 2654435761) mod capacity, capacity a power of two >= 2 * keywords.
void LaneTables::build_hash() {
  std::unordered_map<int32_t, std::vector<std::pair<int32_t, uint64_t>>> by_kw;
  for (int l = 0; l < n(); l++) {
    auto &v = by_kw[kw[l]];
    bool found = false;
    for (auto &wm : v)
      if (wm.first == word[l]) { wm.second |= 1ull << bit[l]; found = true; break; }
    if (!found) v.push_back({word[l], 1ull << bit[l]});
  }
  int32_t cap = 16;
  while (cap < 2 * (int32_t)by_kw.size()) cap <<= 1;
  h_key.assign(cap, -1);
  h_beg.assign(cap, 0);
  h_cnt.assign(cap, 0);
  e_word.clear();
  e_mask.clear();
  for (auto &kv : by_kw) {
    uint32_t h = ((uint32_t)kv.first * 2654435761u) & (uint32_t)(cap - 1);
    while (h_key[h] != -1) h = (h + 1) & (uint32_t)(cap - 1);
    h_key[h] = kv.first;
    h_beg[h] = (int32_t)e_word.size();
    h_cnt[h] = (int32_t)kv.second.size();
    for (auto &wm : kv.second) { e_word.push_back(wm.first); e_mask.push_back(wm.second); }
  }
}

kws_status QueryTables::build(const kws_graph *g, const std::vector<const QIn *> &qs,
                              const std::vector<Placed> &pl, int Wp) {
  nq = (int)qs.size();
  const int32_t n = g->n;
  mask.resize(nq); word.resize(nq); dmax.resize(nq); nk.resize(nq); kcap.resize(nq); hoff.resize(nq);
  coff.resize(nq); ccap.resize(nq); roff.resize(nq + 1); kdoff.resize(nq); eoff.resize(nq); ecap.resize(nq);
  boff.resize(nq);
  bits.clear(); seed_b.clear(); seed_e.clear();
  nhist = ncand = nslots = nkd = nedge = 0;
  for (int i = 0; i < nq; i++) {
    const QIn &Q = *qs[i];
    mask[i] = pl[i].mask;
    word[i] = pl[i].word;
    dmax[i] = Q.dmax;
    nk[i] = Q.nk;
    kcap[i] = std::min(Q.k, n);
    hoff[i] = (int32_t)nhist;
    nhist += Q.nk * Q.dmax + 1;
    ccap[i] = kcap[i] <= 2048 ? kcap[i] : pow2ceil(kcap[i]);
    coff[i] = (int32_t)ncand;
    ncand += ccap[i];
    roff[i] = (int32_t)nslots;
    nslots += kcap[i];
    kdoff[i] = (int32_t)nkd;
    nkd += (int64_t)kcap[i] * Q.nk;
    ecap[i] = Q.nk * Q.dmax;
    eoff[i] = (int32_t)nedge;
    nedge += (int64_t)kcap[i] * ecap[i];
    boff[i] = (int32_t)bits.size();
    for (int j = 0; j < Q.nk; j++) {
      bits.push_back(pl[i].bits[j]);
      const int32_t t = Q.kw[j], key = g->pre[t];
      seed_b.push_back(g->h_inv_ptr[key]);
      seed_e.push_back(g->h_inv_ptr[key + g->span[t]]);
    }
  }
  roff[nq] = (int32_t)nslots;
  if (nhist > INT32_MAX / 2 || ncand > INT32_MAX / 2 || nedge > INT32_MAX / 2 || nkd > INT32_MAX / 2)
    return fail(KWS_EOVERFLOW, "batch too large for one pass");
  wq_ptr.assign(Wp + 1, 0);
  wq.assign(nq, 0);
  for (int i = 0; i < nq; i++) wq_ptr[word[i] + 1]++;
  for (int j = 0; j < Wp; j++) wq_ptr[j + 1] += wq_ptr[j];
  std::vector<int32_t> fill(wq_ptr.begin(), wq_ptr.end() - 1);
  for (int i = 0; i < nq; i++) wq[fill[word[i]]++] = i;
  // one entry more than queries (all zero), so that the score loop can load
  // the entry after a word's last query without a bound check
  qw.assign(nq + 1, QWord{0, 0, 0, 0, 0});
  for (int i = 0; i < nq; i++) {
    const int q = wq[i];
    qw[i] = QWord{mask[q], hoff[q], q, dmax[q], 0};
  }
  // chunks of about 1024 vertices (the select step scans whole chunks for
  // the few that hold a selected root), as long as the histograms (one
  // int per chunk and histogram bin) stay within 512 MB
  const int64_t hist_cap = std::max<int64_t>(1, ((int64_t)1 << 27) / std::max<int64_t>(1, nhist));
  chunks = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n + 1023) / 1024, hist_cap));
  CH = (int)align_up((size_t)((n + chunks - 1) / chunks), 64);
  chunks = (n + CH - 1) / CH;
  // the score step's LDS histogram packs two 16-bit bins per word: the
  // queries from the first whose bins start at or past the middle go to
  // the high halves, so that each query's bins lie in one half
  hist_split = (int32_t)nhist;
  for (int i = 0; i < nq; i++)
    if (2 * (int64_t)hoff[i] >= nhist) { hist_split = hoff[i]; break; }
  hist_words = std::max<int32_t>(hist_split, (int32_t)nhist - hist_split);
  // two copies of it (and, counting te, a sum per query) in at most 64 KB
  hist_lds = (size_t)nq * 8 + (size_t)hist_words * 8 <= 65536;
  te_lds = hist_lds;
  if ((size_t)chunks * (size_t)nhist > (size_t)INT32_MAX) return fail(KWS_EOVERFLOW, "histogram too large");
  return KWS_OK;
}

size_t PlanWriter::add(const void *src, size_t bytes) {
  size = align_up(size, 256);
  const size_t off = size;
  size += std::max<size_t>(bytes, 8);
  pieces.push_back({off, src, bytes});
  return off;
}

kws_status PlanWriter::prepare(Engine &E) {
  // grown to a power of two (at least 64 KB), so that batches whose plans
  // differ a little keep the buffer, and with it the descriptors' device
  // addresses a captured graph was recorded with
  size_t cap = (size_t)64 << 10;
  while (cap < size) cap <<= 1;
  if (E.io().plan.bytes < size) {
    KWS_TRY(E.io().h_plan.ensure(cap, "plan (host)"));
    KWS_TRY(E.io().plan.ensure(cap, "plan"));
  }
  KWS_TRY(E.io().h_plan.ensure(size, "plan (host)"));
  return KWS_OK;
}

void PlanWriter::put(Engine &E, size_t off, const void *src, size_t bytes) {
  std::memcpy(E.io().h_plan.as<uint8_t>() + off, src, bytes);
}

kws_status PlanWriter::upload(Engine &E, hipStream_t s) {
  KWS_TRY(prepare(E));
  uint8_t *hp = E.io().h_plan.as<uint8_t>();
  for (const Piece &p : pieces)
    if (p.bytes && p.src) std::memcpy(hp + p.off, p.src, p.bytes);
  KWS_HIP(hipMemcpyAsync(E.io().plan.p, hp, size, hipMemcpyHostToDevice, s));
  return KWS_OK;
}

QueryOffsets add_query_tables(PlanWriter &pw, const QueryTables &Q) {
  QueryOffsets o;
  const size_t nq = (size_t)Q.nq;
  o.mask = pw.add(Q.mask.data(), nq * 8);
  o.word = pw.add(Q.word.data(), nq * 4);
  o.dmax = pw.add(Q.dmax.data(), nq * 4);
  o.nk = pw.add(Q.nk.data(), nq * 4);
  o.kcap = pw.add(Q.kcap.data(), nq * 4);
  o.hoff = pw.add(Q.hoff.data(), nq * 4);
  o.coff = pw.add(Q.coff.data(), nq * 4);
  o.ccap = pw.add(Q.ccap.data(), nq * 4);
  o.roff = pw.add(Q.roff.data(), (nq + 1) * 4);
  o.kdoff = pw.add(Q.kdoff.data(), nq * 4);
  o.eoff = pw.add(Q.eoff.data(), nq * 4);
  o.ecap = pw.add(Q.ecap.data(), nq * 4);
  o.boff = pw.add(Q.boff.data(), nq * 4);
  o.seed_b = pw.add(Q.seed_b.data(), Q.seed_b.size() * 4);
  o.seed_e = pw.add(Q.seed_e.data(), Q.seed_e.size() * 4);
  o.wq_ptr = pw.add(Q.wq_ptr.data(), Q.wq_ptr.size() * 4);
  o.wq = pw.add(Q.wq.data(), Q.wq.size() * 4);
  o.qw = pw.add(Q.qw.data(), Q.qw.size() * sizeof(QWord));
  o.bits = pw.add(Q.bits.data(), Q.bits.size());
  return o;
}

LaneOffsets add_lane_tables(PlanWriter &pw, LaneTables &L) {
  L.build_hash();
  LaneOffsets o;
  o.seed_off = pw.add(L.seed_off.data(), L.seed_off.size() * 8);
  o.seed_begin = pw.add(L.seed_begin.data(), L.seed_begin.size() * 4);
  o.word = pw.add(L.word.data(), L.word.size() * 4);
  o.bit = pw.add(L.bit.data(), L.bit.size() * 4);
  o.h_key = pw.add(L.h_key.data(), L.h_key.size() * 4);
  o.h_beg = pw.add(L.h_beg.data(), L.h_beg.size() * 4);
  o.h_cnt = pw.add(L.h_cnt.data(), L.h_cnt.size() * 4);
  o.e_word = pw.add(L.e_word.data(), L.e_word.size() * 4);
  o.e_mask = pw.add(L.e_mask.data(), L.e_mask.size() * 8);
  return o;
}

ArenaLayout arena_layout(const QueryTables &Q, size_t extra_bytes, size_t live_words, size_t stats_words) {
  ArenaLayout a;
  Layout l;
  a.extra = l.add(extra_bytes + stats_words * 8);
  a.te = l.add((size_t)Q.nq * 8);
  a.early = l.add((size_t)Q.nq * 8);     // early-termination counts and stop levels
  a.zero_end = align_up(l.size, 8);
  a.nroots = l.add((size_t)Q.nq * 4);
  a.roots = l.add((size_t)Q.nslots * 4);
  a.scores = l.add((size_t)Q.nslots * 4);
  a.ecount = l.add((size_t)Q.nslots * 4);
  a.kwdist = l.add((size_t)Q.nkd);
  a.edges = l.add((size_t)Q.nedge * 8);
  a.size = align_up(l.size, 8);
  Layout z;
  a.z_live = z.add(live_words * 8);
  a.z_stats = a.z_live;   // statistics live in the arena's extra area
  a.z_ccnt = z.add((size_t)Q.nq * 4);
  a.z_wcnt = z.add(4);
  a.z_hist = z.add((size_t)Q.chunks * (size_t)Q.nhist * 4);
  a.z_size = align_up(z.size, 8);
  return a;
}

// seed by vertex when scattering would cost more random atomics than one
// pass over the vertices and their labels
bool seeds_by_vertex(const kws_graph *g, const LaneTables &L) {
  const int mode = g->opt.seed_mode;
  const int64_t lab_total = g->h_lab_total;
  return L.n() > 0 && (mode == 2 || (mode == 0 && L.seed_off.back() > (int64_t)g->n + lab_total * (1 + g->type_depth)));
}

// the table pays when the walks it replaces (one per vertex label) climb a
// type hierarchy, its own walks (one per type) are few against them, and
// it stays small against a state array; a flat label is one hash probe,
// cheaper than building the table
bool type_rows_wanted(const kws_graph *g) {
  const int o = g->opt.seed_table;
  return o > 0 || (o == 0 && g->type_depth > 0 &&
                   8 * (int64_t)g->n_labels <= std::min<int64_t>(g->n, g->h_lab_total));
}

void fill_pass(Pass &P, kws_graph *g, Engine &E, int T, int tiles, int B, const LaneTables &L,
               const LaneOffsets &lo, const QueryTables &Q, const QueryOffsets &qo, const ArenaLayout &al) {
  std::memset(&P, 0, sizeof(P));
  P.n = g->n;
  P.T = T;
  P.tiles = tiles;
  P.Wp = tiles * T;
  P.W = P.Wp;
  P.B = B;
  P.nq = Q.nq;
  P.n_lanes = L.n();
  P.chunks = Q.chunks;
  P.CH = Q.CH;
  P.nhist = (int32_t)Q.nhist;
  P.hist_lds = Q.hist_lds;
  P.hist_split = Q.hist_split;
  P.hist_words = Q.hist_words;
  P.te_lds = Q.te_lds;
  P.force_dir = g->opt.direction;
  P.count_te = g->opt.count_te > 0;
  P.alpha = g->opt.alpha;
  P.total_seeds = L.seed_off.back();
  P.n_hub = g->n_hub;
  P.total_slots = Q.nslots;
  P.total_kd = Q.nkd;
  for (int b = 0; b <= BIN_COUNT; b++) P.bin_begin[b] = g->bin_begin[b];
  P.pstride = (size_t)g->n * P.Wp;
  P.fwd_ptr = g->fwd_ptr; P.fwd_col = g->fwd_col; P.rev_ptr = g->rev_ptr; P.rev_col = g->rev_col;
  P.inv_vtx = g->inv_vtx; P.bin_vtx = g->bin_vtx; P.hub_v = g->hub_v; P.hub_b = g->hub_b; P.hub_e = g->hub_e;
  P.hub_vtx = g->hub_vtx; P.zero_vtx = g->zero_vtx; P.n_hubv = g->n_hubv; P.n_zero = g->n_zero;
  P.vis = E.vis.as<uint64_t>(); P.fr0 = E.fr0.as<uint64_t>(); P.fr1 = E.fr1.as<uint64_t>();
  P.nxt = E.nxt.as<uint64_t>(); P.planes = E.planes.as<uint64_t>();
  P.flist = E.flist.as<int32_t>(); P.flist_eoff = E.flist_eoff.as<int32_t>();
  const uint8_t *dp = E.io().plan.as<uint8_t>();
  P.lane_seed_off = (const int64_t *)(dp + lo.seed_off);
  P.lane_seed_begin = (const int32_t *)(dp + lo.seed_begin);
  P.lane_word = (const int32_t *)(dp + lo.word);
  P.lane_bit = (const int32_t *)(dp + lo.bit);
  P.hcap = (int32_t)L.h_key.size();
  P.h_key = (const int32_t *)(dp + lo.h_key);
  P.h_beg = (const int32_t *)(dp + lo.h_beg);
  P.h_cnt = (const int32_t *)(dp + lo.h_cnt);
  P.e_word = (const int32_t *)(dp + lo.e_word);
  P.e_mask = (const uint64_t *)(dp + lo.e_mask);
  P.lab_ptr = g->lab_ptr;
  P.lab = g->lab;
  P.tparent = g->tparent;
  P.seed_by_vertex = seeds_by_vertex(g, L);
  if (P.seed_by_vertex) P.total_seeds = 0;
  // the type-row table, when wanted and the caller has sized it for Wp
  const size_t tr_bytes = (size_t)g->n_labels * (size_t)P.Wp * 8;
  if (P.seed_by_vertex && type_rows_wanted(g) && E.type_rows.p && E.type_rows.bytes >= tr_bytes) {
    P.type_rows = E.type_rows.as<uint64_t>();
    P.n_types = g->n_labels;
  }
  // vertices per block round of the vertex seeding: rows of Wp + 1 words in
  // at most 64 KB of LDS
  P.seed_vb = BLOCK;
  // rows of Wp + 1 words, plus the live lanes and one flag per vertex of
  // the fused level-0 seeding, within 64 KB of LDS
  while (P.seed_vb > 1 && ((size_t)P.seed_vb * (size_t)(P.Wp + 1) + (size_t)P.Wp) * 8 + (size_t)P.seed_vb * 4 > 65536)
    P.seed_vb >>= 1;
  P.q_mask = (const uint64_t *)(dp + qo.mask);
  P.q_word = (const int32_t *)(dp + qo.word);
  P.q_dmax = (const int32_t *)(dp + qo.dmax);
  P.q_nk = (const int32_t *)(dp + qo.nk);
  P.q_kcap = (const int32_t *)(dp + qo.kcap);
  P.q_hoff = (const int32_t *)(dp + qo.hoff);
  P.q_coff = (const int32_t *)(dp + qo.coff);
  P.q_ccap = (const int32_t *)(dp + qo.ccap);
  P.q_roff = (const int32_t *)(dp + qo.roff);
  P.q_kdoff = (const int32_t *)(dp + qo.kdoff);
  P.q_eoff = (const int32_t *)(dp + qo.eoff);
  P.q_ecap = (const int32_t *)(dp + qo.ecap);
  P.q_boff = (const int32_t *)(dp + qo.boff);
  P.qk_seed_b = (const int32_t *)(dp + qo.seed_b);
  P.qk_seed_e = (const int32_t *)(dp + qo.seed_e);
  P.word_q_ptr = (const int32_t *)(dp + qo.wq_ptr);
  P.word_q = (const int32_t *)(dp + qo.wq);
  P.qw = (const QWord *)(dp + qo.qw);
  P.bits = dp + qo.bits;
  uint8_t *ar = E.io().arena.as<uint8_t>();
  uint8_t *zr = E.io().zero_region.as<uint8_t>();
  P.zero0 = (uint64_t *)ar;
  P.zero0_words = (int64_t)(al.zero_end / 8);
  P.zero1 = (uint64_t *)zr;
  P.zero1_words = (int64_t)(al.z_size / 8);
  P.te = (uint64_t *)(ar + al.te);
  P.early_cnt = (int32_t *)(ar + al.early);
  P.early_stop = P.early_cnt + Q.nq;
  P.cand_cnt = (int32_t *)(zr + al.z_ccnt);
  P.work_cnt = (int32_t *)(zr + al.z_wcnt);
  P.hist = (int32_t *)(zr + al.z_hist);
  P.qsel = E.io().qsel.as<int32_t>();
  P.work = E.io().work.as<int4>();
  P.cand = E.io().cand.as<uint64_t>();
  P.r_nroots = (int32_t *)(ar + al.nroots);
  P.r_roots = (int32_t *)(ar + al.roots);
  P.r_scores = (int32_t *)(ar + al.scores);
  P.r_ecount = (int32_t *)(ar + al.ecount);
  P.r_kwdist = ar + al.kwdist;
  P.r_edges = (int2 *)(ar + al.edges);
}

kws_status collect_results(const QueryTables &Q, const std::vector<const QIn *> &qs, const uint8_t *ha,
                           const ArenaLayout &al, bool te_counted, kws_result *const *out, FlatOut *flat) {
  const uint64_t *h_te = (const uint64_t *)(ha + al.te);
  const int32_t *h_nroots = (const int32_t *)(ha + al.nroots);
  const int32_t *h_roots = (const int32_t *)(ha + al.roots);
  const int32_t *h_scores = (const int32_t *)(ha + al.scores);
  const int32_t *h_ecount = (const int32_t *)(ha + al.ecount);
  const uint8_t *h_kwdist = ha + al.kwdist;
  const int2 *h_edges = (const int2 *)(ha + al.edges);
  for (int i = 0; i < Q.nq; i++) {
    const QIn &qi = *qs[i];
    const int nr = h_nroots[i];
    if (flat) {
      FlatOut &F = *flat;
      F.kw.insert(F.kw.end(), qi.kw, qi.kw + qi.nk);
      F.kw_ptr.push_back((int64_t)F.kw.size());
      F.roots.insert(F.roots.end(), h_roots + Q.roff[i], h_roots + Q.roff[i] + nr);
      F.scores.insert(F.scores.end(), h_scores + Q.roff[i], h_scores + Q.roff[i] + nr);
      F.root_ptr.push_back((int64_t)F.roots.size());
      F.kw_dist.insert(F.kw_dist.end(), h_kwdist + Q.kdoff[i], h_kwdist + Q.kdoff[i] + (size_t)nr * qi.nk);
      F.dist_ptr.push_back((int64_t)F.kw_dist.size());
      for (int j = 0; j < nr; j++) {
        const int c = h_ecount[Q.roff[i] + j];
        const int2 *src = h_edges + Q.eoff[i] + (size_t)j * Q.ecap[i];
        for (int t = 0; t < c; t++) { F.edge_src.push_back(src[t].x); F.edge_dst.push_back(src[t].y); }
        F.edge_ptr.push_back((int64_t)F.edge_src.size());
      }
      F.te.push_back(te_counted ? (int64_t)h_te[i] : -1);
      continue;
    }
    kws_result &r = *out[i];
    std::memset(&r, 0, sizeof(r));
    r.n_roots = nr;
    r.n_kw = qi.nk;
    r.te = te_counted ? (int64_t)h_te[i] : -1;
    int64_t ne = 0;
    for (int j = 0; j < nr; j++) ne += h_ecount[Q.roff[i] + j];
    r.kw = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max(1, qi.nk));
    r.roots = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max(1, nr));
    r.scores = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max(1, nr));
    r.kw_dist = (uint8_t *)malloc((size_t)std::max(1, nr * qi.nk));
    r.edge_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr + 1));
    r.edge_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, ne));
    r.edge_dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(1, ne));
    if (!r.kw || !r.roots || !r.scores || !r.kw_dist || !r.edge_ptr || !r.edge_src || !r.edge_dst) {
      kws_result_free(&r);
      return fail(KWS_ENOMEM, "host result allocation");
    }
    std::memcpy(r.kw, qi.kw, sizeof(int32_t) * (size_t)qi.nk);
    if (nr) {
      std::memcpy(r.roots, h_roots + Q.roff[i], sizeof(int32_t) * (size_t)nr);
      std::memcpy(r.scores, h_scores + Q.roff[i], sizeof(int32_t) * (size_t)nr);
      std::memcpy(r.kw_dist, h_kwdist + Q.kdoff[i], (size_t)nr * qi.nk);
    }
    r.edge_ptr[0] = 0;
    int64_t pos = 0;
    for (int j = 0; j < nr; j++) {
      const int c = h_ecount[Q.roff[i] + j];
      const int2 *src = h_edges + Q.eoff[i] + (size_t)j * Q.ecap[i];
      for (int t = 0; t < c; t++) { r.edge_src[pos] = src[t].x; r.edge_dst[pos] = src[t].y; pos++; }
      r.edge_ptr[j + 1] = pos;
    }
  }
  return KWS_OK;
}

kws_status ensure_state(Engine &E, size_t words_per_array, int planes, hipStream_t s) {
  planes = std::max(planes, 1);
  if (words_per_array <= E.state_words && planes <= E.state_planes) return KWS_OK;
  // a pipelined batch may still use the old arrays
  if (E.vis.p) (void)hipDeviceSynchronize();
  words_per_array = std::max(words_per_array, E.state_words);
  planes = std::max(planes, E.state_planes);
  const size_t b = words_per_array * sizeof(uint64_t);
  E.vis.release(); E.fr0.release(); E.fr1.release(); E.nxt.release(); E.planes.release();
  E.state_words = 0;
  E.state_planes = 0;
  KWS_TRY(E.vis.ensure(b, "vis"));
  KWS_TRY(E.fr0.ensure(b, "frontier"));
  KWS_TRY(E.fr1.ensure(b, "frontier"));
  KWS_TRY(E.nxt.ensure(b, "next"));
  KWS_TRY(E.planes.ensure((size_t)planes * b, "distance planes"));
  KWS_TRY(launch_fill_zero(E.nxt.as<uint64_t>(), words_per_array, s));
  E.state_words = words_per_array;
  E.state_planes = planes;
  return KWS_OK;
}

// Widest useful tile up to max_tile: pull gathers one 8T-byte piece per edge
// and tile, and a miss moves a whole 128-byte line; the streaming kernels
// touch every padded word of every vertex.
int choose_tile(int W, int max_tile, int64_t n, int64_t m) {
  int T = 1;
  double best = 0;
  for (int t = 1; t <= std::max(1, max_tile); t <<= 1) {
    const double tl = (W + t - 1) / t;
    // an edge gathered in a tile costs its column index plus at least one
    // 128-byte cache line of frontier words; every tile word costs about
    // 48 bytes of streaming per vertex (finalize and score)
    const double cost = (double)m * tl * (4.0 + std::max(8.0 * t, 128.0)) + (double)n * tl * t * 8.0 * 3.0 * 2.0;
    if (t == 1 || cost <= best) { best = cost; T = t; }
  }
  return T;
}

}  // namespace kws
