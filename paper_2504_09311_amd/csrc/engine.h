// Host-side planning shared by the batched path and the server (internal):
// query normalisation, lane packing, the per-pass tables uploaded to the
// device, the result arena and the unpacking of results.
#pragma once

#include <array>
#include <vector>

#include "pass.h"

namespace kws {

// A validated query: distinct keywords in ascending order.
struct QIn {
  int32_t nk = 0, dmax = 0, k = 0;
  int32_t kw[KWS_MAX_KW];
};
kws_status normalize_query(const kws_graph *g, const kws_query &q, int idx, QIn &out);

// One lane: the BFS of keyword kw with radius dmax, bit `bit` of word `word`.
struct LaneInfo { int32_t kw, dmax, word, bit; };

// Where a query's keywords sit: its word and the bit of each keyword.
struct Placed {
  int32_t word = 0;
  uint64_t mask = 0;
  std::array<uint8_t, KWS_MAX_KW> bits{};
};

// Lanes of queries [qa, qb) packed into fresh words (see pack_queries).
struct Packing {
  std::vector<LaneInfo> lanes;
  std::vector<int32_t> word_used;
  std::vector<Placed> placed;
  int32_t lane_slots = 0;
};
void pack_queries(const std::vector<QIn> &qs, int qa, int qb, bool share, Packing &pk);

// Seed tables of the lanes a pass starts: slice of the inverted index per lane.
struct LaneTables {
  std::vector<int64_t> seed_off{0};
  std::vector<int32_t> seed_begin, word, bit, kw;
  // keyword hash for seeding by vertex (built by build_hash)
  std::vector<int32_t> h_key, h_beg, h_cnt, e_word;
  std::vector<uint64_t> e_mask;
  void add(const kws_graph *g, const LaneInfo &li);
  void build_hash();
  int n() const { return (int)word.size(); }
};

// Per-query tables of the queries a pass finishes.
struct QueryTables {
  int nq = 0;
  std::vector<uint64_t> mask;
  std::vector<int32_t> word, dmax, nk, kcap, hoff, coff, ccap, roff, kdoff, eoff, ecap, boff;
  std::vector<int32_t> seed_b, seed_e, wq_ptr, wq;
  std::vector<QWord> qw;
  std::vector<uint8_t> bits;
  int64_t nhist = 0, ncand = 0, nslots = 0, nkd = 0, nedge = 0;
  int32_t chunks = 1, CH = 64;
  int32_t hist_split = 0, hist_words = 0;   // score's packed LDS histogram (see k_score)
  bool hist_lds = true, te_lds = true;
  kws_status build(const kws_graph *g, const std::vector<const QIn *> &qs, const std::vector<Placed> &pl, int Wp);
};

// Collects host arrays into the pinned plan buffer and uploads them at once.
struct PlanWriter {
  struct Piece { size_t off; const void *src; size_t bytes; };
  std::vector<Piece> pieces;
  size_t size = 0;
  size_t add(const void *src, size_t bytes);
  // A slot written later with put() (the pass and step descriptors, which
  // hold device addresses of the plan itself).
  size_t reserve(size_t bytes) { return add(nullptr, bytes); }
  // Sizes both copies of the plan buffer, so dev() addresses are final.
  kws_status prepare(Engine &E);
  void put(Engine &E, size_t off, const void *src, size_t bytes);
  kws_status upload(Engine &E, hipStream_t s);
  template <class T> const T *dev(const Engine &E, size_t off) const {
    return (const T *)(E.io().plan.as<uint8_t>() + off);
  }
};

// Result arena (one device buffer, one copy back) and zeroed counters.
struct ArenaLayout {
  size_t te = 0, early = 0, nroots = 0, roots = 0, scores = 0, ecount = 0, kwdist = 0, edges = 0, extra = 0, size = 0;
  size_t zero_end = 0;              // [0, zero_end) is cleared by the seed kernel
  size_t z_live = 0, z_stats = 0, z_ccnt = 0, z_wcnt = 0, z_hist = 0, z_size = 0;
};
ArenaLayout arena_layout(const QueryTables &Q, size_t extra_bytes, size_t live_words, size_t stats_words);

// What finishing an enqueued pass needs: its I/O set, query tables, result
// layout and the shape figures for the batch statistics.
struct PassRecord {
  int io = 0;
  std::vector<const QIn *> qp;
  QueryTables Q;
  ArenaLayout al;
  bool te_counted = false;
  int nq = 0, lanes = 0, lane_slots = 0, W = 0, Wp = 0, tiles = 0, T = 0, D = 0, direction = 0;
  bool early = false, fused = false, seed_table = false;
  float alpha = 0.f;
};

// A submitted batch: its normalized queries and either an enqueued pass or,
// when the batch needs several passes, results computed at submission.
struct AsyncBatch {
  std::vector<QIn> in;
  PassRecord rec;
  bool done = false;
  FlatOut result;
};

// Offsets of the query tables inside the plan buffer.
struct QueryOffsets {
  size_t mask, word, dmax, nk, kcap, hoff, coff, ccap, roff, kdoff, eoff, ecap, boff, seed_b, seed_e, wq_ptr,
      wq, qw, bits;
};
QueryOffsets add_query_tables(PlanWriter &pw, const QueryTables &Q);

// Offsets of the lane seed tables inside the plan buffer.
struct LaneOffsets { size_t seed_off, seed_begin, word, bit, h_key, h_beg, h_cnt, e_word, e_mask; };
LaneOffsets add_lane_tables(PlanWriter &pw, LaneTables &L);

// Seeding by vertex for this batch's lanes (seed_mode, or its auto rule).
bool seeds_by_vertex(const kws_graph *g, const LaneTables &L);
// Whether seeding by vertex goes through the type-row table (seed_table).
bool type_rows_wanted(const kws_graph *g);

// Fills the parts of a Pass common to batch and serving (graph, state,
// lane and query tables, arena, counters); the caller sets the options.
void fill_pass(Pass &P, kws_graph *g, Engine &E, int T, int tiles, int B, const LaneTables &L,
               const LaneOffsets &lo, const QueryTables &Q, const QueryOffsets &qo, const ArenaLayout &al);

// Turns the copied-back arena into results for the pass's queries.
kws_status collect_results(const QueryTables &Q, const std::vector<const QIn *> &qs, const uint8_t *ha,
                           const ArenaLayout &al, bool te_counted, kws_result *const *out, FlatOut *flat);

// Per-vertex search state of `words_per_array` words (nxt starts at zero).
// Search state for words_per_array words per array and `planes` distance
// planes (grows only; nxt is zeroed whenever the arrays are reallocated).
kws_status ensure_state(Engine &E, size_t words_per_array, int planes, hipStream_t s);

// Tile width for W words: gathered 64-byte lines per edge against streamed words.
int choose_tile(int W, int max_tile, int64_t n, int64_t m);

}  // namespace kws
