// Internal declarations of the keyword-search library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kws.h"

namespace kws {
struct AsyncBatch;

// ---------------------------------------------------------------- errors
kws_status fail(kws_status st, const char *fmt, ...);
void clear_error();

#define KWS_HIP(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::kws::fail(KWS_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                            \
  } while (0)

#define KWS_TRY(expr)                       \
  do {                                      \
    kws_status s_ = (expr);                 \
    if (s_ != KWS_OK) return s_;            \
  } while (0)

// ---------------------------------------------------------------- memory
void *dev_alloc(size_t bytes);   // hooks or hipMalloc; nullptr on failure
void dev_free(void *p);

// A device buffer that only grows.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  kws_status ensure(size_t want, const char *what);
  void release();
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// A pinned host buffer that only grows.
struct HostBuf {
  void *p = nullptr;
  size_t bytes = 0;
  kws_status ensure(size_t want, const char *what);
  void release();
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------- profiling
enum KernelClass {
  KC_SEED = 0, KC_PUSH, KC_PULL, KC_FINALIZE, KC_SCORE, KC_THRESHOLD, KC_SELECT,
  KC_FINISH, KC_ANSWER, KC_EXPORT, KC_BUILD, KC_EARLY,
  // host phases of a batch (wall time): planning and plan upload, kernel
  // enqueue, waiting for the device, unpacking the results
  KC_HOST_PLAN, KC_HOST_LAUNCH, KC_HOST_WAIT, KC_HOST_COLLECT, KC_COUNT
};
const char *kernel_class_name(int id);

struct Profiler {
  bool on = false;
  uint64_t mask = ~0ull;                // classes bracketed by events
  struct Pending { int cls; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[KC_COUNT] = {};
  double total_ms[KC_COUNT] = {};
  hipEvent_t get();
  void begin(int cls, hipStream_t s, hipEvent_t *a);
  void end(int cls, hipStream_t s, hipEvent_t a);
  kws_status collect();   // after the stream is synchronised
  void host(int cls, double ms) { if (on) { launches[cls]++; total_ms[cls] += ms; } }
  void reset();
  void release();
};

// ---------------------------------------------------------------- pull bins
// Vertices are grouped by out-degree so each group of threads gets a row of
// a size it handles well. Hub rows are cut into fixed-size edge chunks that
// merge their partial OR with atomics.
enum { BIN_SMALL = 0, BIN_MEDIUM, BIN_LARGE, BIN_COUNT };
constexpr int32_t BIN_SMALL_MAX = 8;
constexpr int32_t BIN_MEDIUM_MAX = 128;
constexpr int32_t BIN_LARGE_MAX = 1024;
constexpr int32_t HUB_CHUNK = 1024;

constexpr int MAX_WORDS = 1024;      // words per device pass (65536 lanes)
constexpr int STAT_STRIPES = 32;     // frontier statistics: stripes of STAT_STRIDE words
constexpr int STAT_STRIDE = 16;      // one 128-byte line per stripe
constexpr int STAT_WORDS = STAT_STRIPES * STAT_STRIDE;
constexpr int BLOCK = 256;

// ---------------------------------------------------------------- engine state
struct Engine {
  // search state, layout [tile][vertex][T words], sized for the largest pass
  DevBuf vis, fr0, fr1, nxt, planes;   // planes: [4][tiles][n][T]
  size_t state_words = 0;              // words per array currently allocated (n * Wp)
  int state_planes = 0;                // distance planes currently allocated
  DevBuf flist, flist_eoff;            // frontier list and in-edge offsets
  DevBuf flags;                        // [2][n] frontier flags (current, next)
  DevBuf flags_tile;                   // [tiles][n] per-tile flags of a fused pulled level
  DevBuf type_rows;                    // [n_labels][Wp] lanes each type starts (table seeding)
  // Buffers of one pass in flight. Set 0 serves the synchronous calls; sets
  // 1 and 2 the two batches a caller may have submitted and not collected.
  struct IoSet {
    DevBuf plan;                       // per-pass plan (device copy)
    DevBuf zero_region;                // per-pass counters zeroed by the seed kernel
    DevBuf qsel;                       // per-query top-k threshold
    DevBuf work;                       // select work items
    DevBuf cand;                       // top-k candidates
    DevBuf arena;                      // results (one D2H copy)
    HostBuf h_plan, h_arena;
    hipEvent_t done = nullptr;         // recorded after the result copy
    void release();
  };
  static constexpr int IO_SETS = 3;
  IoSet ios[IO_SETS];
  int cur = 0;                         // the set the pass being planned uses
  IoSet &io() { return ios[cur]; }
  const IoSet &io() const { return ios[cur]; }
  void release();
};

// graph-capture cache entry
struct GraphEntry {
  std::vector<int64_t> key;
  hipGraphExec_t exec = nullptr;
};

}  // namespace kws

struct kws_graph {
  int device = 0;
  int32_t n = 0;
  int64_t m = 0;
  int32_t n_labels = 0;
  bool hier = false;
  // device graph store
  int32_t *fwd_ptr = nullptr, *fwd_col = nullptr;
  int32_t *rev_ptr = nullptr, *rev_col = nullptr;
  int32_t *inv_ptr = nullptr, *inv_vtx = nullptr;    // by preorder key
  int32_t *lab_ptr = nullptr, *lab = nullptr;        // vertex labels (seeding by vertex)
  int32_t *tparent = nullptr;                        // type parents, or null for flat labels
  int32_t *bin_vtx = nullptr;                        // vertices of the pull bins
  int32_t *hub_v = nullptr, *hub_b = nullptr, *hub_e = nullptr;
  int64_t bin_begin[kws::BIN_COUNT + 1] = {};
  int64_t n_hub = 0;
  int32_t *hub_vtx = nullptr;                        // distinct vertices of the hub chunks
  int32_t *zero_vtx = nullptr;                       // vertices without out-edges
  int64_t n_hubv = 0, n_zero = 0;
  // host mirrors used for planning
  std::vector<int32_t> pre, span;                    // type preorder key and subtree size
  std::vector<int32_t> h_inv_ptr;                    // [n_labels + 1]
  int64_t h_lab_total = 0;                           // number of (vertex, label) pairs
  int32_t type_depth = 0;                            // longest parent chain (0 for flat labels)
  int32_t max_out = 0, max_in = 0;
  int64_t device_bytes = 0;
  // execution
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  std::mutex mu;
  kws_options opt{};
  kws::Engine eng;
  kws::Profiler prof;
  kws_batch_stats last{};
  std::vector<kws::GraphEntry> graphs;
  int64_t graph_captures = 0, graph_replays = 0;     // passes captured / replayed in graph mode
  std::map<int64_t, kws::AsyncBatch *> pending;      // submitted, not yet collected batches
  int64_t next_ticket = 1;
  size_t mem_budget = 0;                             // bytes allowed for search state
};

namespace kws {
// Growing flat output of a batch (turned into a kws_batch_result at the end).
struct FlatOut {
  std::vector<int64_t> root_ptr{0}, kw_ptr{0}, dist_ptr{0}, edge_ptr{0};
  std::vector<int32_t> roots, scores, kw, edge_src, edge_dst;
  std::vector<uint8_t> kw_dist;
  std::vector<int64_t> te;
};
kws_status load_graph(const kws_graph_desc *d, kws_graph **out);
void free_graph(kws_graph *g);
void default_options(kws_options *o);
kws_status search(kws_graph *g, const kws_query *qs, int32_t nq, kws_result *out, FlatOut *flat = nullptr);
kws_status submit_batch(kws_graph *g, const kws_query *qs, int32_t nq, int64_t *ticket);
kws_status collect_batch(kws_graph *g, int64_t ticket, FlatOut *flat);
void drop_pending(kws_graph *g);
kws_status debug_distances(kws_graph *g, int32_t kw, int32_t d_max, uint8_t *dist);
}  // namespace kws
