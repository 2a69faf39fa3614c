// Serving: continuous batching of keyword queries over a resident graph.
//
// The device state is a fixed set of word slots (64 lanes each, state
// memory n * 8 bytes per array per slot). A device step:
//   1. admits waiting queries into free slots (lanes shared inside a slot
//      for equal keyword and d_max);
//   2. seeds the slots filled in this step;
//   3. expands every slot admitted earlier by one level (slot-specific
//      level and lane masks), and finalizes all occupied slots;
//   4. scores, ranks and answers the queries of slots that reached their
//      radius, copies those results back and frees the slots.
// Slots are taken lowest-index first so the occupied words stay in the
// first tiles, and a step only touches the tiles that hold occupied words.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "engine.h"

namespace kws {
namespace {

using Clock = std::chrono::steady_clock;

enum TicketState { T_QUEUED = 0, T_ACTIVE, T_DONE, T_CANCELLED, T_FAILED };

struct Ticket {
  QIn q;
  int state = T_QUEUED;
  bool cancel_requested = false;
  kws_status error = KWS_OK;
  kws_result res{};
  Clock::time_point t_submit, t_done;
};

struct SlotQuery {
  uint64_t ticket;
  QIn q;            // copied at admission: the worker never reads the ticket map unlocked
  Placed placed;
};

struct Slot {
  bool busy = false;
  bool fresh = false;   // filled in the current step (seeded, not expanded yet)
  int level = -1;       // distance of the frontier the slot holds
  int dmax = 0;         // largest radius of its lanes
  std::vector<LaneInfo> lanes;   // word = slot index
  std::vector<SlotQuery> queries;
};

}  // namespace
}  // namespace kws

struct kws_server {
  kws_graph *g = nullptr;
  kws_server_opts opt{};
  kws::Engine eng;
  kws::Profiler prof;
  hipStream_t stream = nullptr;
  int T = 8, tiles_alloc = 1, words = 1, B = 4;
  std::vector<kws::Slot> slots;
  kws::DevBuf live, stats;        // [2][Wp] and [2][STAT_WORDS], ping-pong across steps
  int64_t step_no = 0;

  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  kws_status fatal = KWS_OK;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, kws::Ticket> tickets;
  uint64_t next_ticket = 1;
  // statistics
  int64_t submitted = 0, completed = 0, cancelled = 0, rejected = 0, steps = 0;
  double words_sum = 0;
  std::vector<double> lat_us;
  bool have_first = false;
  kws::Clock::time_point t_first, t_last;
};

namespace kws {
namespace {

// Fills free slots from the queue (FIFO; a slot is closed once the head of
// the queue does not fit it). Called with the lock held.
void admit(kws_server *s) {
  for (size_t si = 0; si < s->slots.size() && !s->queue.empty(); si++) {
    Slot &sl = s->slots[si];
    if (sl.busy) continue;
    int used = 0;
    std::vector<std::array<int32_t, 3>> have;   // (kw, dmax, bit)
    while (!s->queue.empty()) {
      const uint64_t tk = s->queue.front();
      auto it = s->tickets.find(tk);
      if (it == s->tickets.end() || it->second.state != T_QUEUED) { s->queue.pop_front(); continue; }
      const QIn &Q = it->second.q;
      int need = 0;
      for (int j = 0; j < Q.nk; j++) {
        bool found = false;
        for (auto &h : have)
          if (h[0] == Q.kw[j] && h[1] == Q.dmax) { found = true; break; }
        need += !found;
      }
      if (used + need > 64) break;
      SlotQuery sq;
      sq.ticket = tk;
      sq.q = Q;
      sq.placed.word = (int32_t)si;
      for (int j = 0; j < Q.nk; j++) {
        int bit = -1;
        for (auto &h : have)
          if (h[0] == Q.kw[j] && h[1] == Q.dmax) { bit = h[2]; break; }
        if (bit < 0) {
          bit = used++;
          have.push_back({Q.kw[j], Q.dmax, bit});
          sl.lanes.push_back({Q.kw[j], Q.dmax, (int32_t)si, bit});
        }
        sq.placed.bits[j] = (uint8_t)bit;
        sq.placed.mask |= 1ull << bit;
      }
      sl.dmax = std::max(sl.dmax, Q.dmax);
      sl.queries.push_back(sq);
      it->second.state = T_ACTIVE;
      s->queue.pop_front();
    }
    if (!sl.queries.empty()) {
      sl.busy = true;
      sl.fresh = true;
      sl.level = -1;
    }
  }
}

// One device step over the occupied slots. Called without the lock; the
// slot vectors are only touched by the worker thread.
kws_status device_step(kws_server *s, std::vector<std::pair<uint64_t, kws_result>> &done_out) {
  kws_graph *g = s->g;
  Engine &E = s->eng;
  const int n = g->n, T = s->T;
  int top = -1;
  for (size_t i = 0; i < s->slots.size(); i++)
    if (s->slots[i].busy) top = (int)i;
  if (top < 0) return KWS_OK;
  const int tiles = top / T + 1, Wp = tiles * T;

  LaneTables L;
  std::vector<uint64_t> act_exp(Wp, 0), act_new(Wp, 0), act_nn(Wp, 0);
  std::vector<int8_t> newlvl(Wp, 1);
  std::vector<const QIn *> qp;
  std::vector<Placed> placed;
  std::vector<uint64_t> qtickets;
  bool any_expand = false;
  for (int j = 0; j < Wp; j++) {
    if (j >= (int)s->slots.size() || !s->slots[j].busy) continue;
    Slot &sl = s->slots[j];
    const int nl = sl.fresh ? 0 : sl.level + 1;   // distance assigned in this step
    newlvl[j] = (int8_t)nl;
    for (const LaneInfo &li : sl.lanes) {
      const uint64_t bit = 1ull << li.bit;
      if (sl.fresh) L.add(g, li);
      if (li.dmax >= nl) act_new[j] |= bit;
      if (!sl.fresh && li.dmax >= nl) act_exp[j] |= bit;
      if (li.dmax >= nl + 1) act_nn[j] |= bit;
    }
    any_expand |= act_exp[j] != 0;
    if (nl >= sl.dmax)   // radius reached after this step: finish its queries
      for (const SlotQuery &sq : sl.queries) {
        qp.push_back(&sq.q);
        placed.push_back(sq.placed);
        qtickets.push_back(sq.ticket);
      }
  }
  QueryTables Q;
  KWS_TRY(Q.build(g, qp, placed, Wp));
  const ArenaLayout al = arena_layout(Q, 0, 0, 0);
  KWS_TRY(E.io().arena.ensure(al.size, "result arena"));
  KWS_TRY(E.io().h_arena.ensure(al.size, "result arena (host)"));
  KWS_TRY(E.io().zero_region.ensure(al.z_size, "counters"));
  KWS_TRY(E.io().qsel.ensure(sizeof(int32_t) * 4 * (size_t)Q.nq + 16, "query selection"));
  KWS_TRY(E.io().work.ensure(sizeof(int4) * (size_t)std::max<int64_t>(Q.nslots, 1), "select work"));
  KWS_TRY(E.io().cand.ensure(8 * (size_t)std::max<int64_t>(Q.ncand, 1), "candidates"));

  PlanWriter pw;
  const LaneOffsets lo = add_lane_tables(pw, L);
  const QueryOffsets qo = add_query_tables(pw, Q);
  const size_t o_exp = pw.add(act_exp.data(), Wp * 8), o_new = pw.add(act_new.data(), Wp * 8),
               o_nn = pw.add(act_nn.data(), Wp * 8), o_lvl = pw.add(newlvl.data(), Wp);
  const size_t o_pass = pw.reserve(sizeof(Pass)), o_step = pw.reserve(sizeof(Step));
  KWS_TRY(pw.prepare(E));

  Pass P;
  fill_pass(P, g, E, T, tiles, s->B, L, lo, Q, qo, al);
  P.dev = pw.dev<Pass>(E, o_pass);
  P.W = top + 1;
  P.pstride = (size_t)n * s->tiles_alloc * T;   // planes are laid out for every slot
  const int par = (int)(s->step_no & 1);
  uint64_t *live = s->live.as<uint64_t>(), *stats = s->stats.as<uint64_t>();
  const size_t wstride = (size_t)s->tiles_alloc * T;
  P.zero2 = live + (size_t)(1 - par) * wstride;   // this step's outputs start at zero
  P.zero2_words = Wp;
  Step S;
  std::memset(&S, 0, sizeof(S));
  S.act_exp = pw.dev<uint64_t>(E, o_exp);
  S.live_in = live + (size_t)par * wstride;
  S.st_in = stats + (size_t)par * STAT_WORDS;
  S.fr_cur = par ? P.fr1 : P.fr0;
  S.fr_next = par ? P.fr0 : P.fr1;
  S.flags_cur = E.flags.as<uint8_t>() + (size_t)par * n;
  S.flags_next = E.flags.as<uint8_t>() + (size_t)(1 - par) * n;
  S.act_new = pw.dev<uint64_t>(E, o_new);
  S.act_nn = pw.dev<uint64_t>(E, o_nn);
  S.newlvl = pw.dev<int8_t>(E, o_lvl);
  S.st_out = stats + (size_t)(1 - par) * STAT_WORDS;
  S.live_out = live + (size_t)(1 - par) * wstride;
  S.build_list = 1;
  S.write_next = 1;
  S.clear_planes = 1;   // a slot's word stops at its own d_max
  S.dev = pw.dev<Step>(E, o_step);
  pw.put(E, o_pass, &P, sizeof(Pass));
  pw.put(E, o_step, &S, sizeof(Step));
  KWS_TRY(pw.upload(E, s->stream));
  // the step's output statistics are cleared with the counters
  KWS_HIP(hipMemsetAsync(S.st_out, 0, STAT_WORDS * sizeof(uint64_t), s->stream));
  KWS_TRY(launch_seed(P, s->stream, s->prof));
  if (any_expand) KWS_TRY(launch_expand(P, S, s->stream, s->prof));
  KWS_TRY(launch_finalize(P, S, s->stream, s->prof));
  if (Q.nq) {
    KWS_TRY(launch_finish(P, s->stream, s->prof));
    KWS_HIP(hipMemcpyAsync(E.io().h_arena.p, E.io().arena.p, al.size, hipMemcpyDeviceToHost, s->stream));
  }
  KWS_HIP(hipStreamSynchronize(s->stream));
  s->step_no++;
  if (Q.nq) {
    std::vector<kws_result> res(Q.nq);
    std::vector<kws_result *> outs(Q.nq);
    for (int i = 0; i < Q.nq; i++) outs[i] = &res[i];
    KWS_TRY(collect_results(Q, qp, E.io().h_arena.as<uint8_t>(), al, P.count_te != 0, outs.data(), nullptr));
    for (int i = 0; i < Q.nq; i++) done_out.push_back({qtickets[i], res[i]});
  }
  // advance the slots
  for (int j = 0; j < Wp && j < (int)s->slots.size(); j++) {
    Slot &sl = s->slots[j];
    if (!sl.busy) continue;
    sl.level = sl.fresh ? 0 : sl.level + 1;
    sl.fresh = false;
    if (sl.level >= sl.dmax) {
      sl.busy = false;
      sl.lanes.clear();
      sl.queries.clear();
      sl.dmax = 0;
      sl.level = -1;
    }
  }
  return KWS_OK;
}

void worker_loop(kws_server *s) {
  hipSetDevice(s->g->device);
  for (;;) {
    int active = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto busy = [&] {
        for (auto &sl : s->slots)
          if (sl.busy) return true;
        return false;
      };
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || busy(); });
      if (s->fatal == KWS_OK) admit(s);
      for (auto &sl : s->slots) active += sl.busy;
      if (active == 0 && s->stop) break;
      if (active == 0) continue;
    }
    std::vector<std::pair<uint64_t, kws_result>> done;
    kws_status st = device_step(s, done);
    std::lock_guard<std::mutex> lk(s->mu);
    s->steps++;
    s->words_sum += active;
    const auto now = Clock::now();
    for (auto &d : done) {
      auto it = s->tickets.find(d.first);
      if (it == s->tickets.end() || it->second.cancel_requested) {
        kws_result_free(&d.second);
        if (it != s->tickets.end()) it->second.state = T_CANCELLED;
        continue;
      }
      it->second.res = d.second;
      it->second.state = T_DONE;
      it->second.t_done = now;
      s->completed++;
      s->lat_us.push_back(std::chrono::duration<double, std::micro>(now - it->second.t_submit).count());
      s->t_last = now;
    }
    if (st != KWS_OK) {
      // the device state can no longer be trusted: fail everything in flight
      s->fatal = st;
      for (auto &sl : s->slots) {
        for (auto &sq : sl.queries) {
          auto it = s->tickets.find(sq.ticket);
          if (it != s->tickets.end() && it->second.state == T_ACTIVE) {
            it->second.state = T_FAILED;
            it->second.error = st;
          }
        }
        sl = Slot();
      }
      for (uint64_t tk : s->queue) {
        auto it = s->tickets.find(tk);
        if (it != s->tickets.end()) { it->second.state = T_FAILED; it->second.error = st; }
      }
      s->queue.clear();
    }
    s->cv_done.notify_all();
  }
}

}  // namespace
}  // namespace kws

extern "C" {

kws_status kws_server_create(kws_graph *g, const kws_server_opts *opts, kws_server **out) {
  kws::clear_error();
  if (!g || !out) return kws::fail(KWS_EINVAL, "null argument");
  *out = nullptr;
  kws_server_opts o{};
  if (opts) o = *opts;
  if (o.max_dmax < 0 || o.max_dmax > KWS_MAX_DMAX) return kws::fail(KWS_EINVAL, "max_dmax outside 0..%d", KWS_MAX_DMAX);
  if (o.max_dmax == 0) o.max_dmax = KWS_MAX_DMAX;
  if (o.queue_capacity < 0 || o.max_words < 0 || o.mem_bytes < 0) return kws::fail(KWS_EINVAL, "negative option");
  if (o.queue_capacity == 0) o.queue_capacity = 65536;
  if (o.tile_words != 0 && o.tile_words != 1 && o.tile_words != 2 && o.tile_words != 4 && o.tile_words != 8 && o.tile_words != 16)
    return kws::fail(KWS_EINVAL, "tile_words must be 1, 2, 4, 8 or 16");
  int B = 0;
  while ((1 << B) <= o.max_dmax) B++;
  // state arrays per word, and the type-row table's column of the word
  const bool table = kws::type_rows_wanted(g);
  const size_t per_word = (size_t)g->n * 8 * (4 + B) + (table ? (size_t)g->n_labels * 8 : 0);
  const size_t budget = o.mem_bytes ? (size_t)o.mem_bytes : g->mem_budget;
  int words = (int)std::min<size_t>(kws::MAX_WORDS, budget / std::max<size_t>(per_word, 1));
  if (o.max_words) words = std::min(words, o.max_words);
  if (words < 1) return kws::fail(KWS_ENOMEM, "memory budget holds no word slot (%zu bytes per slot)", per_word);
  o.max_words = words;
  // default tile: the widest power of two the slots fill, up to one
  // 128-byte line of words per vertex (a pull gather moves a whole line);
  // a wider tile would pad the state past the memory budget
  if (o.tile_words == 0) o.tile_words = words >= 16 ? 16 : words >= 8 ? 8 : words >= 4 ? 4 : words >= 2 ? 2 : 1;
  // whole tiles only, within the budget (a tile wider than the slots is the
  // caller's explicit choice)
  if (words >= o.tile_words) words = words / o.tile_words * o.tile_words;
  o.max_words = words;
  kws_server *s = new kws_server();
  s->g = g;
  s->opt = o;
  s->T = o.tile_words;
  s->B = B;
  s->words = words;
  s->tiles_alloc = (words + s->T - 1) / s->T;
  s->slots.resize((size_t)words);
  auto bail = [&](kws_status st) {
    s->eng.release();
    s->live.release();
    s->stats.release();
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return st;
  };
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
    return bail(kws::fail(KWS_EDEVICE, "stream creation failed"));
  const size_t wp_alloc = (size_t)s->tiles_alloc * s->T;
  kws_status st = kws::ensure_state(s->eng, (size_t)g->n * wp_alloc, B, s->stream);
  if (st == KWS_OK) st = s->eng.flist.ensure(sizeof(int32_t) * (size_t)g->n, "frontier list");
  if (st == KWS_OK) st = s->eng.flist_eoff.ensure(sizeof(int32_t) * (size_t)g->n, "frontier offsets");
  if (st == KWS_OK) st = s->eng.flags.ensure(2 * (size_t)g->n, "frontier flags");
  if (st == KWS_OK) st = s->live.ensure(2 * wp_alloc * 8, "live lanes");
  if (st == KWS_OK) st = s->stats.ensure(2 * kws::STAT_WORDS * 8, "step statistics");
  if (st == KWS_OK && table) st = s->eng.type_rows.ensure((size_t)g->n_labels * wp_alloc * 8, "type-row table");
  if (st == KWS_OK && hipMemsetAsync(s->live.p, 0, 2 * wp_alloc * 8, s->stream) != hipSuccess)
    st = kws::fail(KWS_EDEVICE, "clearing server state failed");
  if (st == KWS_OK && hipMemsetAsync(s->stats.p, 0, 2 * kws::STAT_WORDS * 8, s->stream) != hipSuccess)
    st = kws::fail(KWS_EDEVICE, "clearing server state failed");
  if (st == KWS_OK && hipStreamSynchronize(s->stream) != hipSuccess)
    st = kws::fail(KWS_EDEVICE, "server set-up failed");
  if (st != KWS_OK) return bail(st);
  s->worker = std::thread(kws::worker_loop, s);
  *out = s;
  return KWS_OK;
}

kws_status kws_server_submit(kws_server *s, const kws_query *q, uint64_t *ticket) {
  kws::clear_error();
  if (!s || !q || !ticket) return kws::fail(KWS_EINVAL, "null argument");
  kws::Ticket t;
  KWS_TRY(kws::normalize_query(s->g, *q, 0, t.q));
  if (t.q.dmax > s->opt.max_dmax) return kws::fail(KWS_EINVAL, "d_max %d above the server's %d", t.q.dmax, s->opt.max_dmax);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return kws::fail(KWS_EINVAL, "server is shutting down");
  if (s->fatal != KWS_OK) return kws::fail(s->fatal, "server stopped after a device error");
  if ((int64_t)s->queue.size() >= s->opt.queue_capacity) {
    s->rejected++;
    return kws::fail(KWS_EBUSY, "admission queue full (%d queries)", s->opt.queue_capacity);
  }
  t.t_submit = kws::Clock::now();
  if (!s->have_first) { s->have_first = true; s->t_first = t.t_submit; }
  const uint64_t id = s->next_ticket++;
  s->tickets.emplace(id, t);
  s->queue.push_back(id);
  s->submitted++;
  *ticket = id;
  s->cv_work.notify_one();
  return KWS_OK;
}

static kws_status take_locked(kws_server *s, uint64_t ticket, kws_result *out, int32_t *done) {
  *done = 0;
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return kws::fail(KWS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  kws::Ticket &t = it->second;
  if (t.state == kws::T_DONE) {
    *out = t.res;
    *done = 1;
    s->tickets.erase(it);
    return KWS_OK;
  }
  if (t.state == kws::T_CANCELLED) {
    s->tickets.erase(it);
    return kws::fail(KWS_ECANCELLED, "ticket %llu was cancelled", (unsigned long long)ticket);
  }
  if (t.state == kws::T_FAILED) {
    const kws_status e = t.error;
    s->tickets.erase(it);
    return kws::fail(e, "ticket %llu failed on the device", (unsigned long long)ticket);
  }
  return KWS_OK;
}

kws_status kws_server_poll(kws_server *s, uint64_t ticket, kws_result *out, int32_t *done) {
  kws::clear_error();
  if (!s || !out || !done) return kws::fail(KWS_EINVAL, "null argument");
  memset(out, 0, sizeof(*out));
  std::lock_guard<std::mutex> lk(s->mu);
  return take_locked(s, ticket, out, done);
}

kws_status kws_server_wait(kws_server *s, uint64_t ticket, int64_t timeout_us, kws_result *out, int32_t *done) {
  kws::clear_error();
  if (!s || !out || !done) return kws::fail(KWS_EINVAL, "null argument");
  memset(out, 0, sizeof(*out));
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] {
    auto it = s->tickets.find(ticket);
    return it == s->tickets.end() || it->second.state >= kws::T_DONE;
  };
  if (timeout_us < 0) s->cv_done.wait(lk, ready);
  else s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  return take_locked(s, ticket, out, done);
}

kws_status kws_server_cancel(kws_server *s, uint64_t ticket) {
  kws::clear_error();
  if (!s) return kws::fail(KWS_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return kws::fail(KWS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  kws::Ticket &t = it->second;
  if (t.state == kws::T_QUEUED) {
    t.state = kws::T_CANCELLED;
    s->cancelled++;
  } else if (t.state == kws::T_ACTIVE) {
    t.cancel_requested = true;
    s->cancelled++;
  } else if (t.state == kws::T_DONE) {
    kws_result_free(&t.res);
    t.state = kws::T_CANCELLED;
    s->cancelled++;
  }
  s->cv_done.notify_all();
  return KWS_OK;
}

kws_status kws_server_stats_get(kws_server *s, kws_server_stats *st) {
  if (!s || !st) return kws::fail(KWS_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(st, 0, sizeof(*st));
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->cancelled = s->cancelled;
  st->rejected = s->rejected;
  st->steps = s->steps;
  st->queued = (int32_t)s->queue.size();
  for (auto &sl : s->slots) st->active_words += sl.busy;
  st->max_words = s->words;
  if (s->completed && s->have_first)
    st->elapsed_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
  st->qps = st->elapsed_s > 0 ? (double)s->completed / st->elapsed_s : 0.0;
  if (!s->lat_us.empty()) {
    std::vector<double> v = s->lat_us;
    auto pct = [&](double p) {
      const size_t k = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
      std::nth_element(v.begin(), v.begin() + (long)k, v.end());
      return v[k];
    };
    st->p50_us = pct(0.50);
    st->p99_us = pct(0.99);
  }
  st->mean_active_words = s->steps ? s->words_sum / (double)s->steps : 0.0;
  return KWS_OK;
}

void kws_server_destroy(kws_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (uint64_t tk : s->queue) {
      auto it = s->tickets.find(tk);
      if (it != s->tickets.end() && it->second.state == kws::T_QUEUED) it->second.state = kws::T_CANCELLED;
    }
    s->queue.clear();
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &kv : s->tickets)
    if (kv.second.state == kws::T_DONE) kws_result_free(&kv.second.res);
  s->eng.release();
  s->live.release();
  s->stats.release();
  s->prof.release();
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
