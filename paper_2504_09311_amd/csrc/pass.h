// Device-side descriptors of one device pass and of one BFS step, and the
// launchers of the kernels that work on them (internal).
//
// Lanes. Every (query, keyword) needs one BFS. A lane is one bit of a 64-bit
// mask word; all lanes of a query sit in one word, and queries packed into
// the same word share a lane when they ask for the same keyword with the
// same d_max. Per vertex and word the device keeps:
//   vis    lanes whose BFS has reached the vertex (dist <= current level)
//   fr     lanes that reached it exactly at the current level (two buffers)
//   nxt    lanes arriving at the next level (push target; zero between steps)
//   P_b    bit b of the distance of each reached lane (bit-sliced distances)
// Layout [tile][vertex][T words]: the T words of one vertex are contiguous,
// so one neighbour visit gathers 8*T bytes; a tile is one contiguous slab.
#pragma once

#include <vector>

#include "kws_internal.h"

namespace kws {

// What the score step reads of one query, in word order (queries of word j
// at [word_q_ptr[j], word_q_ptr[j + 1])): uniform across a wavefront, so
// its fields come in through scalar loads.
struct QWord {
  uint64_t mask;       // the query's lanes in its word
  int32_t hoff;        // its histogram's offset in a chunk's histogram
  int32_t q;           // query index in the pass
  int32_t dmax;
  int32_t pad;
};

struct Pass {
  const Pass *dev;                   // where this descriptor lives in device memory (kernels read it there)
  int32_t graph_mode;                // launch grids depend on the pass shape only (captured graphs replay)
  // sizes
  int32_t n, T, tiles, Wp, B, nq, n_lanes;
  int32_t W;                         // words in use; words W..Wp-1 pad the last tile (no lane, no query)
  int32_t chunks, CH, nhist, hist_lds, te_lds;
  int32_t hist_split, hist_words;    // score's LDS histogram: first bin of the high halves, words per copy
  int32_t force_dir, count_te;
  float alpha;
  int64_t total_seeds, n_hub, total_slots, total_kd;
  int64_t bin_begin[BIN_COUNT + 1];
  size_t pstride;                    // words per plane = tiles * n * T
  // graph
  const int32_t *fwd_ptr, *fwd_col, *rev_ptr, *rev_col, *inv_vtx;
  const int32_t *bin_vtx, *hub_v, *hub_b, *hub_e;
  const int32_t *hub_vtx, *zero_vtx;   // distinct hub vertices; vertices without out-edges
  int64_t n_hubv, n_zero;
  // state
  uint64_t *vis, *fr0, *fr1, *nxt, *planes;
  int32_t *flist, *flist_eoff;
  // lanes to seed: by scattering over inverted-index slices, or (seed_by_vertex)
  // by every vertex looking its labels and their type ancestors up in a hash
  // of keyword -> [(word, lane mask)] entries
  int32_t seed_by_vertex, seed_vb, hcap;   // seed_vb: vertices per block round (power of two <= BLOCK)
  const int32_t *lab_ptr, *lab, *tparent;
  const int32_t *h_key, *h_beg, *h_cnt, *e_word;
  const uint64_t *e_mask;
  // optional type-row table [n_types][Wp]: the lanes each type starts, built
  // from the hash once per pass (k_type_rows); null: walk per vertex label
  uint64_t *type_rows;
  int64_t n_types;
  const int64_t *lane_seed_off;      // [n_lanes + 1]
  const int32_t *lane_seed_begin;    // [n_lanes]
  const int32_t *lane_word, *lane_bit;
  // queries to finish (score, rank, answer)
  const int32_t *word_q_ptr, *word_q;
  const QWord *qw;                   // [nq + 1] in word order, the last entry zero
  const uint64_t *q_mask;
  const int32_t *q_word, *q_dmax, *q_nk, *q_kcap, *q_hoff, *q_coff, *q_ccap, *q_roff, *q_kdoff,
      *q_eoff, *q_ecap, *q_boff;
  const uint8_t *bits;               // lane bit of each query keyword, keyword order
  const int32_t *qk_seed_b, *qk_seed_e;   // inverted-index slice of each query keyword
  // zeroed by the seed kernel
  uint64_t *zero0; int64_t zero0_words;
  uint64_t *zero1; int64_t zero1_words;
  uint64_t *zero2; int64_t zero2_words;
  uint64_t *te;                      // [nq]
  int32_t *cand_cnt, *work_cnt, *hist;
  // scratch
  int32_t *qsel;                     // [nq * 4]: k_eff, s*, need, c_lt
  int4 *work;
  uint64_t *cand;
  // top-k early termination: per query, complete roots scoring at most the
  // current level, and the level after which the query stopped, plus one
  // (0: still running); the plan's lane-activity table [(levels + 2) x Wp],
  // from which the stopped queries' lanes are cleared
  int32_t early, D;
  int32_t *early_cnt, *early_stop;
  uint64_t *act_tab;
  // results
  int32_t *r_nroots, *r_roots, *r_scores, *r_ecount;
  uint8_t *r_kwdist;
  int2 *r_edges;
};

// One BFS step over all words: expand the current frontier (lanes in
// act_exp) and finalize the arrivals. Per word, newlvl is the distance the
// arrivals get; 0 means the word starts here (vis is reset to the seeds and
// the distance planes are cleared).
struct Step {
  const Step *dev;           // where this descriptor lives in device memory
  const uint64_t *act_exp;   // [Wp] lanes that expand in this step
  const uint64_t *live_in;   // [Wp] lanes whose current frontier is non-empty
  const uint64_t *st_in;     // statistics of the current frontier: (n_f << 32 | m_f), m_u, list counter
  const uint64_t *fr_cur;
  uint64_t *fr_next;
  const uint8_t *flags_cur;  // [n] 1 if the vertex is in the frontier being expanded
  uint8_t *flags_next;
  const uint64_t *act_new;   // [Wp] lanes allowed to gain a distance in this step
  const uint64_t *act_nn;    // [Wp] lanes that would expand in the following step
  const int8_t *newlvl;      // [Wp]
  uint64_t *st_out;          // statistics of the new frontier: (n_f << 32 | m_f), m_u
  uint64_t *live_out;        // [Wp]
  int32_t build_list;        // write the frontier list (a following push reads it)
  int32_t write_next;        // write fr_next and live_out
  int32_t next_in_plane;     // the next frontier is distance plane 0 (level 1 of a batched pass, where
                             // plane 0 is stored outright): fr_next is not written, the next step's
                             // fr_cur is the plane
  int32_t clear_planes;      // clear the distance planes when a word starts; otherwise every
                             // word reaches level 2^b for every plane b, where b is stored
  int32_t fused;             // a pulled level is finalized by the pull itself (every word's
                             // newlvl >= 1, planes stored at their first level): k_pull_fin for
                             // the rows, k_fin_list for the hub vertices, k_fin_stats for the
                             // per-vertex flags and statistics; k_finalize then only runs for
                             // pushed or empty levels
  uint8_t *flags_tile;       // [tiles][n] per vertex and tile: bit 0 new lanes, bit 1 lanes still to reach
};

kws_status launch_seed(const Pass &P, hipStream_t s, Profiler &prof);
// Seeding by vertex and the finalize of level 0 in one kernel (batched
// passes: every word starts at level 0; S is the level-0 step).
kws_status launch_seed_level0(const Pass &P, const Step &S, hipStream_t s, Profiler &prof);
kws_status launch_expand(const Pass &P, const Step &S, hipStream_t s, Profiler &prof);
kws_status launch_finalize(const Pass &P, const Step &S, hipStream_t s, Profiler &prof);
// Score, rank and answer; with last, the score kernel also does the
// finalize of that step (the last level of a batched pass).
kws_status launch_finish(const Pass &P, hipStream_t s, Profiler &prof, const Step *last = nullptr);
kws_status launch_export(const Pass &P, uint8_t *out, hipStream_t s);
// Top-k early termination after level L (every level of the pass up to L
// finalized): queries with at least k complete roots scoring at most L stop,
// and lanes no running query needs leave the activity table.
kws_status launch_early(const Pass &P, int L, hipStream_t s, Profiler &prof);
kws_status launch_fill_zero(uint64_t *p, size_t words, hipStream_t s);
// Everything the launches of a pass in graph mode depend on: passes with
// equal keys launch the same kernels with the same grids, LDS sizes and
// arguments, so one captured graph serves them all (fin_last: the score
// kernel finalizes the last level).
void graph_shape_key(const Pass &P, const std::vector<Step> &steps, bool fin_last, std::vector<int64_t> &key);

}  // namespace kws
