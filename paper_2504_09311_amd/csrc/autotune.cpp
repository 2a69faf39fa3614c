// Autotuner: picks tile width, push/pull policy and seeding mode for a graph
// and batch shape by timing a sample batch, and remembers the choice on disk.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"

namespace kws {
namespace {

// Everything the answers contain, for the identical-results check.
bool same_answers(const FlatOut &a, const FlatOut &b) {
  return a.root_ptr == b.root_ptr && a.roots == b.roots && a.scores == b.scores && a.kw == b.kw &&
         a.kw_dist == b.kw_dist && a.edge_ptr == b.edge_ptr && a.edge_src == b.edge_src &&
         a.edge_dst == b.edge_dst && a.te == b.te;
}

std::string shape_key(const kws_graph *g, const kws_query *qs, int nq) {
  int64_t kw = 0;
  int dmax = 0;
  for (int i = 0; i < nq; i++) { kw += qs[i].n_kw; dmax = std::max(dmax, qs[i].d_max); }
  char buf[256];
  snprintf(buf, sizeof(buf), "n=%d m=%lld labels=%d maxout=%d maxin=%d hier=%d nq=%d kw=%lld dmax=%d", g->n,
           (long long)g->m, g->n_labels, g->max_out, g->max_in, g->hier ? 1 : 0, nq, (long long)kw, dmax);
  return buf;
}

bool cache_lookup(const char *path, const std::string &key, kws_options *o) {
  FILE *f = path ? fopen(path, "r") : nullptr;
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char *bar = strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    if (key != line) continue;
    kws_options t;
    default_options(&t);
    if (sscanf(bar + 1, "direction=%d alpha=%f tile_words=%d seed_mode=%d fused_pull=%d early_stop=%d",
               &t.direction, &t.alpha, &t.tile_words, &t.seed_mode, &t.fused_pull, &t.early_stop) >= 3) {
      *o = t;   // the last matching line wins
      found = true;
    }
  }
  fclose(f);
  return found;
}

void cache_store(const char *path, const std::string &key, const kws_options &o, double ms) {
  FILE *f = path ? fopen(path, "a") : nullptr;
  if (!f) return;
  fprintf(f, "%s|direction=%d alpha=%g tile_words=%d seed_mode=%d fused_pull=%d early_stop=%d ms=%.4f\n",
          key.c_str(), o.direction, o.alpha, o.tile_words, o.seed_mode, o.fused_pull, o.early_stop, ms);
  fclose(f);
}

kws_status time_config(kws_graph *g, const kws_query *qs, int nq, int reps, const kws_options &o, double *ms,
                       FlatOut *answers) {
  g->opt = o;
  FlatOut warm;
  KWS_TRY(search(g, qs, nq, nullptr, &warm));
  std::vector<double> t;
  for (int r = 0; r < reps; r++) {
    FlatOut f;
    const auto a = std::chrono::steady_clock::now();
    KWS_TRY(search(g, qs, nq, nullptr, &f));
    t.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count());
  }
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  *answers = std::move(warm);
  return KWS_OK;
}

}  // namespace
}  // namespace kws

extern "C" kws_status kws_autotune(kws_graph *g, const kws_query *qs, int32_t nq, int32_t reps, double budget_ms,
                                   const char *cache_path, kws_options *best, kws_tune_report *report) {
  kws::clear_error();
  if (!g || (!qs && nq > 0) || nq < 1) return kws::fail(KWS_EINVAL, "need a non-empty sample batch");
  if (reps < 1) reps = 3;
  std::lock_guard<std::mutex> lk(g->mu);
  kws_tune_report rep{};
  const kws_options saved = g->opt;
  const std::string key = kws::shape_key(g, qs, nq);
  kws_options choice;
  if (kws::cache_lookup(cache_path, key, &choice)) {
    g->opt = choice;
    g->opt.use_graph = saved.use_graph;
    g->opt.count_te = saved.count_te;
    g->opt.share_lanes = saved.share_lanes;
    rep.from_cache = 1;
    if (best) *best = g->opt;
    if (report) *report = rep;
    return KWS_OK;
  }
  std::vector<kws_options> grid;
  kws_options d;
  kws::default_options(&d);
  d.count_te = saved.count_te;       // what the caller asked the answers to contain stays as it was
  d.share_lanes = saved.share_lanes;
  grid.push_back(d);
  for (int tw : {1, 2, 4, 8, 16})
    for (int pol = 0; pol < 6; pol++) {
      kws_options o = d;
      o.tile_words = tw;
      const float alphas[4] = {0.5f, 2.0f, 8.0f, 32.0f};
      if (pol < 4) { o.direction = 0; o.alpha = alphas[pol]; }
      else o.direction = pol == 4 ? 1 : 2;
      if (o.tile_words == d.tile_words && o.direction == d.direction && o.alpha == d.alpha) continue;
      grid.push_back(o);
    }
  const auto t0 = std::chrono::steady_clock::now();
  kws::FlatOut ref;
  double best_ms = 0;
  kws_options best_o = d;
  kws_status st = KWS_OK;
  const size_t n_main = grid.size();
  for (size_t i = 0; i < grid.size(); i++) {
    double ms = 0;
    kws::FlatOut ans;
    st = kws::time_config(g, qs, nq, reps, grid[i], &ms, &ans);
    if (st != KWS_OK) break;
    rep.configs_tried++;
    if (i == 0) {
      ref = std::move(ans);
      rep.default_ms = ms;
      best_ms = ms;
      best_o = grid[0];
    } else {
      if (!kws::same_answers(ref, ans)) {
        st = kws::fail(KWS_EDEVICE, "autotune: configuration %zu (tile %d, direction %d, alpha %g, seed mode %d) "
                       "changed the answers", i, grid[i].tile_words, grid[i].direction, grid[i].alpha, grid[i].seed_mode);
        break;
      }
      if (ms < best_ms) { best_ms = ms; best_o = grid[i]; }
    }
    const double spent = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (budget_ms > 0 && spent > budget_ms) break;
    if (i + 1 == n_main)
      for (int sm : {1, 2}) {   // second phase: the best so far under each explicit seeding mode
        kws_options o = best_o;
        o.seed_mode = sm;
        grid.push_back(o);
      }
    if (i + 1 == n_main + 2) {   // third phase: the finalize fused into pulls or not; early termination
      for (int fp : {1, -1}) {
        kws_options o = best_o;
        o.fused_pull = fp;
        grid.push_back(o);
      }
      if (!saved.count_te) {     // it changes te (fewer levels scanned), so only when te is not asked for
        kws_options o = best_o;
        o.early_stop = 1;
        grid.push_back(o);
      }
    }
  }
  if (st != KWS_OK) {
    g->opt = saved;
    return st;
  }
  best_o.use_graph = saved.use_graph;
  best_o.count_te = saved.count_te;
  best_o.share_lanes = saved.share_lanes;
  g->opt = best_o;
  rep.best_ms = best_ms;
  kws::cache_store(cache_path, key, best_o, best_ms);
  if (best) *best = best_o;
  if (report) *report = rep;
  return KWS_OK;
}
