// Batched keyword search: plan a device pass, run it (directly or as a
// replayed hipGraph), unpack the results.
//
// A pass seeds every lane (level 0), then for each level l < D expands the
// lanes whose d_max > l and finalizes the arrivals, then scores, ranks and
// answers every query of the pass.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "engine.h"

namespace kws {

namespace {

constexpr kws_status PASS_TOO_WIDE = (kws_status)1;   // internal: retry with fewer queries

bool score_finalizes_last(const Pass &P, const std::vector<Step> &steps);

// Device work of one pass: seed, D levels, finish.
kws_status launch_pass(kws_graph *g, const Pass &P, const std::vector<Step> &steps) {
  hipStream_t s = g->stream;
  if (P.seed_by_vertex) {
    KWS_TRY(launch_seed_level0(P, steps[0], s, g->prof));
  } else {
    KWS_TRY(launch_seed(P, s, g->prof));
    KWS_TRY(launch_finalize(P, steps[0], s, g->prof));
  }
  if (steps.size() > 1) KWS_TRY(launch_early(P, 0, s, g->prof));
  // With tiles of at most 8 words a score thread holds a vertex's whole
  // tile row, so the score kernel does the last level's finalize (its
  // stores fill whole lines); wider tiles keep the separate pass, where the
  // stores of the merge would be scattered partial lines.
  // With the finalize fused into pulled levels the last level may already
  // be final when scoring starts, so the score kernel does not merge it.
  const bool fin_last = score_finalizes_last(P, steps);
  for (size_t i = 1; i < steps.size(); i++) {
    KWS_TRY(launch_expand(P, steps[i], s, g->prof));
    if (i + 1 < steps.size() || !fin_last) KWS_TRY(launch_finalize(P, steps[i], s, g->prof));
    if (i + 1 < steps.size()) KWS_TRY(launch_early(P, (int)i, s, g->prof));
  }
  return launch_finish(P, s, g->prof, fin_last ? &steps.back() : nullptr);
}

// Whether the score kernel finalizes the last level (launch_pass decides
// the same way).
bool score_finalizes_last(const Pass &P, const std::vector<Step> &steps) {
  return steps.size() > 1 && P.T <= 8 && !steps.back().fused;
}

// The same work through a hipGraph captured once per pass shape and
// replayed for every later pass of that shape. The kernels read the pass
// and step descriptors from the plan buffer, which each pass uploads before
// the launch, so the graph holds no per-batch value: its key is the
// descriptors' device addresses and the launch shape (graph_shape_key).
kws_status launch_pass_graph(kws_graph *g, const Pass &P, const std::vector<Step> &steps) {
  std::vector<int64_t> key;
  graph_shape_key(P, steps, score_finalizes_last(P, steps), key);
  for (auto &e : g->graphs)
    if (e.key == key) {
      KWS_HIP(hipGraphLaunch(e.exec, g->stream));
      g->graph_replays++;
      return KWS_OK;
    }
  hipGraph_t graph = nullptr;
  KWS_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
  kws_status st = launch_pass(g, P, steps);
  hipError_t e = hipStreamEndCapture(g->stream, &graph);
  if (st != KWS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
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
  g->graph_captures++;
  KWS_HIP(hipGraphLaunch(exec, g->stream));
  return KWS_OK;
}

// Plans a pass over queries [qa, qb) of qs, uploads its plan and enqueues all
// of its device work and the result copy on the handle's stream, using the
// engine's current I/O set; finish_pass waits for it and unpacks. With
// export_dist, the pass (one keyword) copies its distances out instead.
kws_status enqueue_pass(kws_graph *g, const std::vector<QIn> &qs, int qa, int qb, int max_words,
                        uint8_t *export_dist, PassRecord &rec) {
  const bool export_only = export_dist != nullptr;
  Engine &E = g->eng;
  const kws_options &o = g->opt;
  const int32_t n = g->n;
  const int nq = qb - qa;
  using clk = std::chrono::steady_clock;
  const auto ms_since = [](clk::time_point a) { return std::chrono::duration<double, std::milli>(clk::now() - a).count(); };
  auto t_phase = clk::now();
  Packing pk;
  pack_queries(qs, qa, qb, o.share_lanes >= 0 && !export_only, pk);
  const int W = (int)pk.word_used.size();
  if (W > max_words) return PASS_TOO_WIDE;
  const int T = export_only ? 1 : choose_tile(W, o.tile_words, n, g->m);
  const int tiles = (W + T - 1) / T, Wp = tiles * T;
  int D = 0;
  for (int q = qa; q < qb; q++) D = std::max(D, qs[q].dmax);
  int B = 0;
  while ((1 << B) <= D) B++;
  if (D == 0) B = 0;

  KWS_TRY(ensure_state(E, (size_t)n * Wp, B, g->stream));
  KWS_TRY(E.flist.ensure(sizeof(int32_t) * (size_t)n, "frontier list"));
  KWS_TRY(E.flist_eoff.ensure(sizeof(int32_t) * (size_t)n, "frontier offsets"));
  KWS_TRY(E.flags.ensure(2 * (size_t)n, "frontier flags"));
  // Fusing the finalize into pulled levels pays when the pull's per-row
  // writes are whole 128-byte lines (16-word tiles) and a state array is far
  // larger than the 256 MB Infinity Cache, where the separate finalize pass
  // streams from HBM; with smaller state that pass runs from cache and
  // narrower rows would be scattered partial-line writes.
  const bool fused = D > 0 && (o.fused_pull > 0 || (o.fused_pull == 0 && T == 16 &&
                                                    (size_t)n * (size_t)Wp * 8 > ((size_t)512 << 20)));
  if (fused) KWS_TRY(E.flags_tile.ensure((size_t)n * tiles, "tile flags"));

  LaneTables L;
  for (const LaneInfo &li : pk.lanes) L.add(g, li);
  if (!export_only && type_rows_wanted(g) && seeds_by_vertex(g, L))
    KWS_TRY(E.type_rows.ensure((size_t)g->n_labels * (size_t)Wp * 8, "type-row table"));
  // per level: lanes with d_max >= level, and the distance each level assigns
  std::vector<uint64_t> act((size_t)(D + 2) * Wp, 0);
  for (const LaneInfo &li : pk.lanes)
    for (int lv = 0; lv <= li.dmax; lv++) act[(size_t)lv * Wp + li.word] |= 1ull << li.bit;
  std::vector<int8_t> newlvl((size_t)(D + 1) * Wp);
  for (int lv = 0; lv <= D; lv++) std::fill(newlvl.begin() + (size_t)lv * Wp, newlvl.begin() + (size_t)(lv + 1) * Wp, (int8_t)lv);
  std::vector<const QIn *> &qp = rec.qp;
  qp.resize(nq);
  for (int i = 0; i < nq; i++) qp[i] = &qs[qa + i];
  QueryTables &Q = rec.Q;
  KWS_TRY(Q.build(g, qp, pk.placed, Wp));

  const ArenaLayout al = arena_layout(Q, 0, (size_t)(D + 1) * Wp, (size_t)(D + 1) * STAT_WORDS);
  rec.al = al;
  KWS_TRY(E.io().arena.ensure(al.size, "result arena"));
  KWS_TRY(E.io().h_arena.ensure(al.size, "result arena (host)"));
  KWS_TRY(E.io().zero_region.ensure(al.z_size, "counters"));
  KWS_TRY(E.io().qsel.ensure(sizeof(int32_t) * 4 * (size_t)nq + 16, "query selection"));
  KWS_TRY(E.io().work.ensure(sizeof(int4) * (size_t)std::max<int64_t>(Q.nslots, 1), "select work"));
  KWS_TRY(E.io().cand.ensure(8 * (size_t)std::max<int64_t>(Q.ncand, 1), "candidates"));

  PlanWriter pw;
  // the descriptors first: their device addresses (which a captured graph
  // holds) then do not move with the sizes of the batch's tables
  const size_t o_pass = pw.reserve(sizeof(Pass));
  const size_t o_steps = pw.reserve(sizeof(Step) * (size_t)(D + 1));
  const LaneOffsets lo = add_lane_tables(pw, L);
  const QueryOffsets qo = add_query_tables(pw, Q);
  const size_t o_act = pw.add(act.data(), act.size() * 8);
  const size_t o_lvl = pw.add(newlvl.data(), newlvl.size());
  KWS_TRY(pw.prepare(E));

  const bool graph_mode = o.use_graph > 0 && !g->prof.on && !export_only;
  Pass P;
  fill_pass(P, g, E, T, tiles, B, L, lo, Q, qo, al);
  P.W = W;
  P.dev = pw.dev<Pass>(E, o_pass);
  P.graph_mode = graph_mode;
  // top-k early termination, on request: its per-level check reads every
  // vertex's vis and planes, which on the measured workloads costs more
  // than the expansion it saves
  P.D = D;
  P.act_tab = const_cast<uint64_t *>(pw.dev<uint64_t>(E, o_act));
  P.early = !export_only && nq > 0 && D > 0 && o.early_stop > 0 &&
            nq <= 16384;   // per-query counters in LDS (rounded up to a power of two in graph mode)
  uint64_t *stats = (uint64_t *)(E.io().arena.as<uint8_t>() + al.extra);
  uint64_t *live = (uint64_t *)(E.io().zero_region.as<uint8_t>() + al.z_live);
  const uint64_t *act_d = pw.dev<uint64_t>(E, o_act);
  const int8_t *lvl_d = pw.dev<int8_t>(E, o_lvl);
  std::vector<Step> steps;
  for (int lv = -1; lv < D; lv++) {   // step lv expands level lv (none for lv = -1) into level lv + 1
    Step S;
    std::memset(&S, 0, sizeof(S));
    if (lv >= 0) {
      S.act_exp = act_d + (size_t)(lv + 1) * Wp;
      S.live_in = live + (size_t)lv * Wp;
      S.st_in = stats + (size_t)lv * STAT_WORDS;
      S.fr_cur = (lv & 1) ? P.fr1 : P.fr0;
      S.flags_cur = E.flags.as<uint8_t>() + (size_t)(lv & 1) * n;
    }
    S.fr_next = ((lv + 1) & 1) ? P.fr1 : P.fr0;
    S.flags_next = E.flags.as<uint8_t>() + (size_t)((lv + 1) & 1) * n;
    S.act_new = act_d + (size_t)(lv + 1) * Wp;
    S.act_nn = act_d + (size_t)(lv + 2) * Wp;
    S.newlvl = lvl_d + (size_t)(lv + 1) * Wp;
    S.st_out = stats + (size_t)(lv + 1) * STAT_WORDS;
    S.live_out = live + (size_t)(lv + 1) * Wp;
    S.build_list = S.write_next = lv + 1 < D;
    // level 1's frontier equals distance plane 0, which this step stores
    // outright for every vertex-word (planes are not cleared per word in a
    // batched pass): the next step gathers from the plane and the frontier
    // buffer is not written. Level 2 stores plane 1 outright, so nothing
    // writes plane 0 while it is gathered.
    S.next_in_plane = lv == 0 && S.write_next && B >= 1;
    if (lv == 1 && D >= 2 && B >= 1) S.fr_cur = P.planes;
    S.fused = lv >= 0 && fused;
    S.flags_tile = fused ? E.flags_tile.as<uint8_t>() : nullptr;
    S.dev = pw.dev<Step>(E, o_steps) + (lv + 1);
    steps.push_back(S);
  }
  pw.put(E, o_pass, &P, sizeof(Pass));
  pw.put(E, o_steps, steps.data(), sizeof(Step) * steps.size());
  KWS_TRY(pw.upload(E, g->stream));

  if (export_only) {
    DevBuf tmp;
    KWS_TRY(tmp.ensure((size_t)n, "distance export"));
    kws_status st = launch_pass(g, P, steps);
    if (st == KWS_OK) st = launch_export(P, tmp.as<uint8_t>(), g->stream);
    if (st == KWS_OK && hipMemcpyAsync(export_dist, tmp.p, (size_t)n, hipMemcpyDeviceToHost, g->stream) != hipSuccess)
      st = fail(KWS_EDEVICE, "export copy failed");
    if (st == KWS_OK && hipStreamSynchronize(g->stream) != hipSuccess) st = fail(KWS_EDEVICE, "export sync failed");
    tmp.release();
    return st;
  }

  g->prof.host(KC_HOST_PLAN, ms_since(t_phase));
  t_phase = clk::now();
  if (graph_mode) KWS_TRY(launch_pass_graph(g, P, steps));
  else KWS_TRY(launch_pass(g, P, steps));
  KWS_HIP(hipMemcpyAsync(E.io().h_arena.p, E.io().arena.p, al.size, hipMemcpyDeviceToHost, g->stream));
  if (!E.io().done) KWS_HIP(hipEventCreateWithFlags(&E.io().done, hipEventDisableTiming));
  KWS_HIP(hipEventRecord(E.io().done, g->stream));
  g->prof.host(KC_HOST_LAUNCH, ms_since(t_phase));
  rec.io = E.cur;
  rec.te_counted = P.count_te != 0;
  rec.nq = nq;
  rec.lanes = L.n();
  rec.lane_slots = pk.lane_slots;
  rec.W = W;
  rec.Wp = Wp;
  rec.tiles = tiles;
  rec.T = T;
  rec.D = D;
  rec.direction = o.direction;
  rec.alpha = o.alpha;
  rec.early = P.early != 0;
  rec.fused = fused;
  rec.seed_table = P.type_rows != nullptr;
  return KWS_OK;
}

// Waits for an enqueued pass, unpacks its results (into out[0..nq) or flat)
// and adds its statistics to the handle's last-batch statistics.
kws_status finish_pass(kws_graph *g, PassRecord &rec, kws_result *out, FlatOut *flat) {
  using clk = std::chrono::steady_clock;
  const auto ms_since = [](clk::time_point a) { return std::chrono::duration<double, std::milli>(clk::now() - a).count(); };
  Engine::IoSet &io = g->eng.ios[rec.io];
  auto t_phase = clk::now();
  KWS_HIP(hipEventSynchronize(io.done));
  g->prof.host(KC_HOST_WAIT, ms_since(t_phase));
  t_phase = clk::now();
  KWS_TRY(g->prof.collect());
  const int nq = rec.nq, D = rec.D;
  std::vector<kws_result *> outs(nq);
  for (int i = 0; i < nq; i++) outs[i] = out ? &out[i] : nullptr;
  KWS_TRY(collect_results(rec.Q, rec.qp, io.h_arena.as<uint8_t>(), rec.al, rec.te_counted, outs.data(), flat));
  g->prof.host(KC_HOST_COLLECT, ms_since(t_phase));

  const uint64_t *h_stats = (const uint64_t *)(io.h_arena.as<uint8_t>() + rec.al.extra);
  kws_batch_stats &bs = g->last;
  bs.fused_pull = rec.fused ? 1 : 0;
  if (rec.seed_table) bs.seed_table = 1;
  if (rec.early) {
    const int32_t *h_stop = (const int32_t *)(io.h_arena.as<uint8_t>() + rec.al.early) + nq;
    for (int i = 0; i < nq; i++)
      if (h_stop[i] > 0) {
        bs.early_stopped += 1;
        bs.levels_skipped += rec.qp[i]->dmax - (h_stop[i] - 1);
      }
  }
  bs.queries += nq;
  bs.lanes += rec.lanes;
  bs.lane_slots += rec.lane_slots;
  bs.words += rec.W;
  bs.words_padded += rec.Wp;
  bs.tiles += rec.tiles;
  bs.tile_words = rec.T;
  bs.levels = std::max(bs.levels, D);
  bs.passes += 1;
  for (int lv = 0; lv <= D && lv <= KWS_MAX_DMAX; lv++) {
    uint64_t packed = 0, mu = 0;
    for (int k = 0; k < STAT_STRIPES; k++) {
      packed += h_stats[(size_t)lv * STAT_WORDS + (size_t)k * STAT_STRIDE];
      mu += h_stats[(size_t)lv * STAT_WORDS + (size_t)k * STAT_STRIDE + 1];
    }
    const uint32_t nf = (uint32_t)(packed >> 32), mf = (uint32_t)packed;
    bs.frontier[lv] += nf;
    bs.frontier_edges[lv] += mf;
    bs.unfinished_edges[lv] += (int64_t)mu;
    if (lv == D) break;
    int dir = 0;
    if (nf) dir = (rec.direction == 1 || rec.direction == 2) ? rec.direction
                  : ((double)rec.alpha * mf > (double)mu ? 2 : 1);
    bs.pulled[lv] |= dir == 2;
  }
  return KWS_OK;
}

kws_status run_pass(kws_graph *g, const std::vector<QIn> &qs, int qa, int qb, int max_words, bool export_only,
                    uint8_t *export_dist, kws_result *out, FlatOut *flat) {
  PassRecord rec;
  g->eng.cur = 0;
  kws_status st = enqueue_pass(g, qs, qa, qb, max_words, export_only ? export_dist : nullptr, rec);
  if (st != KWS_OK || export_only) return st;
  return finish_pass(g, rec, out ? out + qa : nullptr, flat);
}

}  // namespace

void default_options(kws_options *o) {
  std::memset(o, 0, sizeof(*o));
  o->direction = 0;
  o->alpha = 8.0f;
  o->tile_words = 16;
  o->block = BLOCK;
  o->use_graph = 0;
  o->share_lanes = 1;
  o->count_te = 0;
  o->fused_pull = 0;
  o->early_stop = 0;
  o->seed_table = 0;
}

namespace {

int max_pass_words(const kws_graph *g) {
  const size_t per_word = (size_t)g->n * 8 * 8;   // vis, 2 frontiers, nxt, 4 planes
  const size_t budget_words = g->mem_budget / std::max<size_t>(per_word, 1);
  return (int)std::max<size_t>(1, std::min<size_t>(MAX_WORDS, budget_words));
}

// Next-fit estimate of the words a batch needs (queries never split).
int estimate_words(const std::vector<QIn> &in) {
  int used = 0, free_in_last = 0;
  for (const QIn &q : in) {
    if (free_in_last >= q.nk) { free_in_last -= q.nk; continue; }
    used++;
    free_in_last = 64 - q.nk;
  }
  return used;
}

}  // namespace

kws_status search(kws_graph *g, const kws_query *qs, int32_t nq, kws_result *out, FlatOut *flat) {
  if (!g || (!qs && nq > 0) || (!out && !flat && nq > 0) || nq < 0) return fail(KWS_EINVAL, "null argument");
  if (out)
    for (int i = 0; i < nq; i++) std::memset(&out[i], 0, sizeof(kws_result));
  std::vector<QIn> in(nq);
  for (int i = 0; i < nq; i++) KWS_TRY(normalize_query(g, qs[i], i, in[i]));
  std::memset(&g->last, 0, sizeof(g->last));
  // split into passes that respect the word and memory limits
  const int max_words = max_pass_words(g);
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

kws_status submit_batch(kws_graph *g, const kws_query *qs, int32_t nq, int64_t *ticket) {
  if (!g || !ticket || (!qs && nq > 0) || nq < 0) return fail(KWS_EINVAL, "null argument");
  *ticket = 0;
  bool held[Engine::IO_SETS] = {};
  int in_flight = 0;
  for (auto &kv : g->pending) {
    in_flight++;
    if (!kv.second->done) held[kv.second->rec.io] = true;
  }
  if (in_flight >= Engine::IO_SETS - 1)
    return fail(KWS_EBUSY, "%d batches submitted and not collected", in_flight);
  int io = 1;
  while (io < Engine::IO_SETS && held[io]) io++;
  AsyncBatch *b = new AsyncBatch();
  b->in.resize(nq);
  for (int i = 0; i < nq; i++) {
    kws_status st = normalize_query(g, qs[i], i, b->in[i]);
    if (st != KWS_OK) { delete b; return st; }
  }
  const int max_words = max_pass_words(g);
  kws_status st = PASS_TOO_WIDE;
  if (nq > 0 && estimate_words(b->in) <= max_words) {
    g->eng.cur = io;
    st = enqueue_pass(g, b->in, 0, nq, max_words, nullptr, b->rec);
    g->eng.cur = 0;
  }
  if (st == PASS_TOO_WIDE) {   // several passes (or none): compute now
    b->done = true;
    st = search(g, qs, nq, nullptr, &b->result);
  }
  if (st != KWS_OK) {
    g->eng.state_words = 0;   // force a clean reallocation (nxt must start at zero)
    delete b;
    return st;
  }
  *ticket = g->next_ticket++;
  g->pending[*ticket] = b;
  return KWS_OK;
}

kws_status collect_batch(kws_graph *g, int64_t ticket, FlatOut *flat) {
  if (!g || !flat) return fail(KWS_EINVAL, "null argument");
  auto it = g->pending.find(ticket);
  if (it == g->pending.end()) return fail(KWS_EINVAL, "no submitted batch with ticket %lld", (long long)ticket);
  AsyncBatch *b = it->second;
  g->pending.erase(it);
  kws_status st = KWS_OK;
  std::memset(&g->last, 0, sizeof(g->last));
  if (b->done) *flat = std::move(b->result);
  else st = finish_pass(g, b->rec, nullptr, flat);
  g->last.queries = (int32_t)b->in.size();
  delete b;
  return st;
}

void drop_pending(kws_graph *g) {
  for (auto &kv : g->pending) delete kv.second;
  g->pending.clear();
}

}  // namespace kws
