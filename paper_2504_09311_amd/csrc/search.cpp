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

// Device work of one pass: seed, D levels, finish.
kws_status launch_pass(kws_graph *g, const Pass &P, const std::vector<Step> &steps) {
  hipStream_t s = g->stream;
  KWS_TRY(launch_seed(P, s, g->prof));
  KWS_TRY(launch_finalize(P, steps[0], s, g->prof));
  for (size_t i = 1; i < steps.size(); i++) {
    KWS_TRY(launch_expand(P, steps[i], s, g->prof));
    KWS_TRY(launch_finalize(P, steps[i], s, g->prof));
  }
  return launch_finish(P, s, g->prof);
}

// The same work through a hipGraph captured once per pass shape (the key
// holds every launch argument) and replayed afterwards.
kws_status launch_pass_graph(kws_graph *g, const Pass &P, const std::vector<Step> &steps) {
  std::vector<uint8_t> key(sizeof(Pass) + steps.size() * sizeof(Step));
  std::memcpy(key.data(), &P, sizeof(Pass));
  std::memcpy(key.data() + sizeof(Pass), steps.data(), steps.size() * sizeof(Step));
  for (auto &e : g->graphs)
    if (e.key == key) {
      KWS_HIP(hipGraphLaunch(e.exec, g->stream));
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
  KWS_HIP(hipGraphLaunch(exec, g->stream));
  return KWS_OK;
}

kws_status run_pass(kws_graph *g, const std::vector<QIn> &qs, int qa, int qb, int max_words, bool export_only,
                    uint8_t *export_dist, kws_result *out, FlatOut *flat) {
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

  KWS_TRY(ensure_state(E, (size_t)n * Wp, g->stream));
  KWS_TRY(E.flist.ensure(sizeof(int32_t) * (size_t)n, "frontier list"));
  KWS_TRY(E.flist_eoff.ensure(sizeof(int32_t) * (size_t)n, "frontier offsets"));
  KWS_TRY(E.flags.ensure(2 * (size_t)n, "frontier flags"));

  LaneTables L;
  for (const LaneInfo &li : pk.lanes) L.add(g, li);
  // per level: lanes with d_max >= level, and the distance each level assigns
  std::vector<uint64_t> act((size_t)(D + 2) * Wp, 0);
  for (const LaneInfo &li : pk.lanes)
    for (int lv = 0; lv <= li.dmax; lv++) act[(size_t)lv * Wp + li.word] |= 1ull << li.bit;
  std::vector<int8_t> newlvl((size_t)(D + 1) * Wp);
  for (int lv = 0; lv <= D; lv++) std::fill(newlvl.begin() + (size_t)lv * Wp, newlvl.begin() + (size_t)(lv + 1) * Wp, (int8_t)lv);
  std::vector<const QIn *> qp(nq);
  for (int i = 0; i < nq; i++) qp[i] = &qs[qa + i];
  QueryTables Q;
  KWS_TRY(Q.build(g, qp, pk.placed, Wp));

  const ArenaLayout al = arena_layout(Q, 0, (size_t)(D + 1) * Wp, (size_t)(D + 1) * STAT_WORDS);
  KWS_TRY(E.arena.ensure(al.size, "result arena"));
  KWS_TRY(E.h_arena.ensure(al.size, "result arena (host)"));
  KWS_TRY(E.zero_region.ensure(al.z_size, "counters"));
  KWS_TRY(E.qsel.ensure(sizeof(int32_t) * 4 * (size_t)nq + 16, "query selection"));
  KWS_TRY(E.work.ensure(sizeof(int4) * (size_t)std::max<int64_t>(Q.nslots, 1), "select work"));
  KWS_TRY(E.cand.ensure(8 * (size_t)std::max<int64_t>(Q.ncand, 1), "candidates"));

  PlanWriter pw;
  const LaneOffsets lo = add_lane_tables(pw, L);
  const QueryOffsets qo = add_query_tables(pw, Q);
  const size_t o_act = pw.add(act.data(), act.size() * 8);
  const size_t o_lvl = pw.add(newlvl.data(), newlvl.size());
  KWS_TRY(pw.upload(E, g->stream));

  Pass P;
  fill_pass(P, g, E, T, tiles, B, L, lo, Q, qo, al);
  P.W = W;
  uint64_t *stats = (uint64_t *)(E.arena.as<uint8_t>() + al.extra);
  uint64_t *live = (uint64_t *)(E.zero_region.as<uint8_t>() + al.z_live);
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
    steps.push_back(S);
  }

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
  if (o.use_graph > 0 && !g->prof.on) KWS_TRY(launch_pass_graph(g, P, steps));
  else KWS_TRY(launch_pass(g, P, steps));
  KWS_HIP(hipMemcpyAsync(E.h_arena.p, E.arena.p, al.size, hipMemcpyDeviceToHost, g->stream));
  g->prof.host(KC_HOST_LAUNCH, ms_since(t_phase));
  t_phase = clk::now();
  KWS_HIP(hipStreamSynchronize(g->stream));
  g->prof.host(KC_HOST_WAIT, ms_since(t_phase));
  t_phase = clk::now();
  KWS_TRY(g->prof.collect());

  std::vector<kws_result *> outs(nq);
  for (int i = 0; i < nq; i++) outs[i] = out ? &out[qa + i] : nullptr;
  KWS_TRY(collect_results(Q, qp, E.h_arena.as<uint8_t>(), al, P.count_te != 0, outs.data(), flat));
  g->prof.host(KC_HOST_COLLECT, ms_since(t_phase));

  const uint64_t *h_stats = (const uint64_t *)(E.h_arena.as<uint8_t>() + al.extra);
  kws_batch_stats &bs = g->last;
  bs.queries += nq;
  bs.lanes += L.n();
  bs.lane_slots += pk.lane_slots;
  bs.words += W;
  bs.words_padded += Wp;
  bs.tiles += tiles;
  bs.tile_words = T;
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
    if (nf) dir = (o.direction == 1 || o.direction == 2) ? o.direction
                  : ((double)o.alpha * mf > (double)mu ? 2 : 1);
    bs.pulled[lv] |= dir == 2;
  }
  return KWS_OK;
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
}

kws_status search(kws_graph *g, const kws_query *qs, int32_t nq, kws_result *out, FlatOut *flat) {
  if (!g || (!qs && nq > 0) || (!out && !flat && nq > 0) || nq < 0) return fail(KWS_EINVAL, "null argument");
  if (out)
    for (int i = 0; i < nq; i++) std::memset(&out[i], 0, sizeof(kws_result));
  std::vector<QIn> in(nq);
  for (int i = 0; i < nq; i++) KWS_TRY(normalize_query(g, qs[i], i, in[i]));
  std::memset(&g->last, 0, sizeof(g->last));
  // split into passes that respect the word and memory limits
  const size_t per_word = (size_t)g->n * 8 * 8;   // vis, 2 frontiers, nxt, 4 planes
  const size_t budget_words = g->mem_budget / std::max<size_t>(per_word, 1);
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
