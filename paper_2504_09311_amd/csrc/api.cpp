// C ABI entry points, error reporting, device/host buffers and the profiler.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "kws_internal.h"

namespace kws {

// ---------------------------------------------------------------- errors
namespace {
thread_local char g_err[1024] = "";
}

kws_status fail(kws_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_err[0] = 0; }

// ---------------------------------------------------------------- memory
namespace {
kws_alloc_fn g_alloc = nullptr;
kws_free_fn g_free = nullptr;
void *g_ctx = nullptr;
std::mutex g_mem_mu;
std::atomic<int64_t> g_dev_bytes{0};
int64_t g_mem_limit = -1;   // KWS_MEM_LIMIT_BYTES, -1 = unlimited
bool g_limit_read = false;
std::mutex g_limit_mu;                          // guards g_mem_limit and g_limit_read
std::vector<std::pair<void *, size_t>> g_live;   // allocations and their sizes

int64_t mem_limit() {
  std::lock_guard<std::mutex> lk(g_limit_mu);
  if (!g_limit_read) {
    const char *e = getenv("KWS_MEM_LIMIT_BYTES");
    g_mem_limit = e ? atoll(e) : -1;
    g_limit_read = true;
  }
  return g_mem_limit;
}
}  // namespace

void set_mem_limit(int64_t bytes) {
  std::lock_guard<std::mutex> lk(g_limit_mu);
  g_mem_limit = bytes < 0 ? -1 : bytes;
  g_limit_read = true;
}

void *dev_alloc(size_t bytes) {
  const int64_t lim = mem_limit();
  std::lock_guard<std::mutex> lk(g_mem_mu);
  if (lim >= 0 && g_dev_bytes.load() + (int64_t)bytes > lim) return nullptr;
  void *p = nullptr;
  if (g_alloc) {
    p = g_alloc(bytes, g_ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    hipGetLastError();
    p = nullptr;
  }
  if (p) {
    g_dev_bytes += (int64_t)bytes;
    g_live.push_back({p, bytes});
  }
  return p;
}

void dev_free(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mem_mu);
  for (size_t i = 0; i < g_live.size(); i++)
    if (g_live[i].first == p) {
      g_dev_bytes -= (int64_t)g_live[i].second;
      g_live[i] = g_live.back();
      g_live.pop_back();
      break;
    }
  if (g_free) g_free(p, g_ctx);
  else hipFree(p);
}

int64_t dev_bytes_in_use() { return g_dev_bytes.load(); }

kws_status DevBuf::ensure(size_t want, const char *what) {
  if (want <= bytes && p) return KWS_OK;
  // a pipelined batch may still read the old buffer
  if (p) (void)hipDeviceSynchronize();
  release();
  size_t b = std::max<size_t>(want, 256);
  p = dev_alloc(b);
  if (!p) return fail(KWS_ENOMEM, "device allocation of %zu bytes for %s failed", b, what);
  bytes = b;
  return KWS_OK;
}

void DevBuf::release() {
  dev_free(p);
  p = nullptr;
  bytes = 0;
}

kws_status HostBuf::ensure(size_t want, const char *what) {
  if (want <= bytes && p) return KWS_OK;
  release();
  size_t b = std::max<size_t>(want, 4096);
  b += b / 4;
  if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
    hipGetLastError();
    p = nullptr;
    return fail(KWS_ENOMEM, "pinned host allocation of %zu bytes for %s failed", b, what);
  }
  bytes = b;
  return KWS_OK;
}

void HostBuf::release() {
  if (p) hipHostFree(p);
  p = nullptr;
  bytes = 0;
}

void Engine::IoSet::release() {
  DevBuf *d[] = {&plan, &zero_region, &qsel, &work, &cand, &arena};
  for (DevBuf *b : d) b->release();
  h_plan.release();
  h_arena.release();
  if (done) (void)hipEventDestroy(done);
  done = nullptr;
}

void Engine::release() {
  DevBuf *d[] = {&vis, &fr0, &fr1, &nxt, &planes, &flist, &flist_eoff, &flags, &flags_tile, &type_rows};
  for (DevBuf *b : d) b->release();
  for (IoSet &x : ios) x.release();
  state_words = 0;
  state_planes = 0;
}

// ---------------------------------------------------------------- profiler
const char *kernel_class_name(int id) {
  static const char *names[KC_COUNT] = {"seed",   "push",      "pull",        "finalize",    "score",
                                        "threshold", "select", "finish",    "answer",      "export",
                                        "build",  "early",     "host_plan",   "host_launch", "host_wait",
                                        "host_collect"};
  return id >= 0 && id < KC_COUNT ? names[id] : nullptr;
}

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::begin(int cls, hipStream_t s, hipEvent_t *a) {
  *a = nullptr;
  if (!on || !((mask >> cls) & 1ull)) return;
  *a = get();
  if (*a) hipEventRecord(*a, s);
}

void Profiler::end(int cls, hipStream_t s, hipEvent_t a) {
  if (!on || !a) return;
  hipEvent_t b = get();
  if (!b) return;
  hipEventRecord(b, s);
  pending.push_back({cls, a, b});
}

kws_status Profiler::collect() {
  // launches of a pipelined batch still on the device stay pending
  std::vector<Pending> later;
  for (auto &p : pending) {
    float ms = 0.f;
    const hipError_t e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e == hipErrorNotReady) {
      later.push_back(p);
      continue;
    }
    if (e == hipSuccess) {
      launches[p.cls]++;
      total_ms[p.cls] += ms;
    }
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.swap(later);
  return KWS_OK;
}

void Profiler::reset() {
  for (int i = 0; i < KC_COUNT; i++) { launches[i] = 0; total_ms[i] = 0; }
}

void Profiler::release() {
  for (auto &p : pending) { pool.push_back(p.a); pool.push_back(p.b); }
  pending.clear();
  for (hipEvent_t e : pool) hipEventDestroy(e);
  pool.clear();
}

}  // namespace kws

template <class T>
static T *copy_out(const std::vector<T> &v) {
  T *p = (T *)malloc(sizeof(T) * std::max<size_t>(1, v.size()));
  if (p && !v.empty()) memcpy(p, v.data(), sizeof(T) * v.size());
  return p;
}

// ================================================================ C ABI
extern "C" {

const char *kws_last_error(void) { return kws::g_err; }

kws_status kws_set_allocator(kws_alloc_fn alloc, kws_free_fn free_, void *ctx) {
  if ((alloc == nullptr) != (free_ == nullptr))
    return kws::fail(KWS_EINVAL, "set both allocator hooks or neither");
  std::lock_guard<std::mutex> lk(kws::g_mem_mu);
  if (!kws::g_live.empty()) return kws::fail(KWS_EBUSY, "device allocations are live; set hooks first");
  kws::g_alloc = alloc;
  kws::g_free = free_;
  kws::g_ctx = ctx;
  return KWS_OK;
}

kws_status kws_set_mem_limit(int64_t bytes) {
  kws::clear_error();
  kws::set_mem_limit(bytes);
  return KWS_OK;
}

int64_t kws_mem_in_use(void) { return kws::dev_bytes_in_use(); }

kws_status kws_load_graph(const kws_graph_desc *desc, kws_graph **out) {
  kws::clear_error();
  kws_status st = kws::load_graph(desc, out);
  if (st != KWS_OK) return st;
  kws_graph *g = *out;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    hipGetLastError();
    free_b = 0;
  }
  size_t budget = (size_t)((double)free_b * 0.85);
  const int64_t lim = kws::mem_limit();
  if (lim >= 0) {
    const int64_t left = lim - kws::dev_bytes_in_use();
    budget = std::min<size_t>(budget ? budget : (size_t)left, (size_t)std::max<int64_t>(left, 0));
  }
  g->mem_budget = budget;
  return KWS_OK;
}

void kws_free_graph(kws_graph *g) { kws::free_graph(g); }

kws_status kws_keyword_search(kws_graph *g, const kws_query *q, kws_result *out) {
  kws::clear_error();
  if (!g || !q || !out) return kws::fail(KWS_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g->mu);
  return kws::search(g, q, 1, out);
}

kws_status kws_search_batch(kws_graph *g, const kws_query *qs, int32_t nq, kws_result *out) {
  kws::clear_error();
  if (!g) return kws::fail(KWS_EINVAL, "null graph");
  std::lock_guard<std::mutex> lk(g->mu);
  return kws::search(g, qs, nq, out);
}

static kws_status flat_to_c(int32_t nq, kws::FlatOut &f, kws_batch_result *out) {
  out->nq = nq;
  out->total_roots = (int64_t)f.roots.size();
  out->root_ptr = copy_out(f.root_ptr);
  out->roots = copy_out(f.roots);
  out->scores = copy_out(f.scores);
  out->kw_ptr = copy_out(f.kw_ptr);
  out->kw = copy_out(f.kw);
  out->dist_ptr = copy_out(f.dist_ptr);
  out->kw_dist = copy_out(f.kw_dist);
  out->edge_ptr = copy_out(f.edge_ptr);
  out->edge_src = copy_out(f.edge_src);
  out->edge_dst = copy_out(f.edge_dst);
  out->te = copy_out(f.te);
  if (!out->root_ptr || !out->roots || !out->scores || !out->kw_ptr || !out->kw || !out->dist_ptr ||
      !out->kw_dist || !out->edge_ptr || !out->edge_src || !out->edge_dst || !out->te) {
    kws_batch_result_free(out);
    return kws::fail(KWS_ENOMEM, "host result allocation");
  }
  return KWS_OK;
}

kws_status kws_search_batch_flat(kws_graph *g, const kws_query *qs, int32_t nq, kws_batch_result *out) {
  kws::clear_error();
  if (!g || !out) return kws::fail(KWS_EINVAL, "null argument");
  memset(out, 0, sizeof(*out));
  kws::FlatOut f;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    kws_status st = kws::search(g, qs, nq, nullptr, &f);
    if (st != KWS_OK) return st;
  }
  return flat_to_c(nq, f, out);
}

kws_status kws_search_batch_submit(kws_graph *g, const kws_query *qs, int32_t nq, int64_t *ticket) {
  kws::clear_error();
  if (!g || !ticket) return kws::fail(KWS_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g->mu);
  return kws::submit_batch(g, qs, nq, ticket);
}

kws_status kws_search_batch_collect(kws_graph *g, int64_t ticket, kws_batch_result *out) {
  kws::clear_error();
  if (!g || !out) return kws::fail(KWS_EINVAL, "null argument");
  memset(out, 0, sizeof(*out));
  kws::FlatOut f;
  int32_t nq = 0;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    kws_status st = kws::collect_batch(g, ticket, &f);
    if (st != KWS_OK) return st;
    nq = g->last.queries;
  }
  return flat_to_c(nq, f, out);
}

void kws_batch_result_free(kws_batch_result *r) {
  if (!r) return;
  free(r->root_ptr); free(r->roots); free(r->scores); free(r->kw_ptr); free(r->kw); free(r->dist_ptr);
  free(r->kw_dist); free(r->edge_ptr); free(r->edge_src); free(r->edge_dst); free(r->te);
  memset(r, 0, sizeof(*r));
}

void kws_result_free(kws_result *r) {
  if (!r) return;
  free(r->kw); free(r->roots); free(r->scores); free(r->kw_dist);
  free(r->edge_ptr); free(r->edge_src); free(r->edge_dst);
  memset(r, 0, sizeof(*r));
}

kws_status kws_debug_distances(kws_graph *g, int32_t kw, int32_t d_max, uint8_t *dist_n) {
  kws::clear_error();
  if (!g) return kws::fail(KWS_EINVAL, "null graph");
  std::lock_guard<std::mutex> lk(g->mu);
  return kws::debug_distances(g, kw, d_max, dist_n);
}

kws_status kws_set_options(kws_graph *g, const kws_options *opt) {
  if (!g || !opt) return kws::fail(KWS_EINVAL, "null argument");
  kws_options o;
  kws::default_options(&o);
  if (opt->direction < 0 || opt->direction > 2) return kws::fail(KWS_EINVAL, "direction must be 0, 1 or 2");
  o.direction = opt->direction;
  if (opt->alpha < 0) return kws::fail(KWS_EINVAL, "alpha must be >= 0");
  if (opt->alpha > 0) o.alpha = opt->alpha;
  if (opt->tile_words) {
    const int t = opt->tile_words;
    if (t != 1 && t != 2 && t != 4 && t != 8 && t != 16) return kws::fail(KWS_EINVAL, "tile_words must be 1, 2, 4, 8 or 16");
    o.tile_words = t;
  }
  if (opt->block && opt->block != kws::BLOCK) return kws::fail(KWS_EINVAL, "block must be %d", kws::BLOCK);
  o.use_graph = opt->use_graph > 0 ? 1 : 0;
  o.share_lanes = opt->share_lanes < 0 ? -1 : 1;
  o.count_te = opt->count_te > 0 ? 1 : 0;
  if (opt->seed_mode < 0 || opt->seed_mode > 2) return kws::fail(KWS_EINVAL, "seed_mode must be 0, 1 or 2");
  o.seed_mode = opt->seed_mode;
  if (opt->fused_pull < -1 || opt->fused_pull > 1) return kws::fail(KWS_EINVAL, "fused_pull must be -1, 0 or 1");
  o.fused_pull = opt->fused_pull;
  if (opt->early_stop < -1 || opt->early_stop > 1) return kws::fail(KWS_EINVAL, "early_stop must be -1, 0 or 1");
  o.early_stop = opt->early_stop;
  if (opt->seed_table < -1 || opt->seed_table > 1) return kws::fail(KWS_EINVAL, "seed_table must be -1, 0 or 1");
  o.seed_table = opt->seed_table;
  std::lock_guard<std::mutex> lk(g->mu);
  g->opt = o;
  return KWS_OK;
}

kws_status kws_get_options(kws_graph *g, kws_options *opt) {
  if (!g || !opt) return kws::fail(KWS_EINVAL, "null argument");
  *opt = g->opt;
  return KWS_OK;
}

kws_status kws_set_stream(kws_graph *g, void *hip_stream) {
  if (!g) return kws::fail(KWS_EINVAL, "null graph");
  std::lock_guard<std::mutex> lk(g->mu);
  if (g->stream) hipStreamSynchronize(g->stream);
  g->stream = hip_stream ? (hipStream_t)hip_stream : g->own_stream;
  return KWS_OK;
}

void *kws_get_stream(kws_graph *g) { return g ? (void *)g->stream : nullptr; }

kws_status kws_graph_info_get(kws_graph *g, kws_graph_info *info) {
  if (!g || !info) return kws::fail(KWS_EINVAL, "null argument");
  info->n = g->n;
  info->m = g->m;
  info->n_labels = g->n_labels;
  info->hierarchical = g->hier ? 1 : 0;
  info->device_bytes = g->device_bytes;
  info->max_out_degree = g->max_out;
  info->max_in_degree = g->max_in;
  info->graph_captures = g->graph_captures;
  info->graph_replays = g->graph_replays;
  return KWS_OK;
}

kws_status kws_profile_enable(kws_graph *g, int32_t on) {
  if (!g) return kws::fail(KWS_EINVAL, "null graph");
  std::lock_guard<std::mutex> lk(g->mu);
  g->prof.on = on != 0;
  return KWS_OK;
}

kws_status kws_profile_classes(kws_graph *g, uint64_t mask) {
  if (!g) return kws::fail(KWS_EINVAL, "null graph");
  std::lock_guard<std::mutex> lk(g->mu);
  g->prof.mask = mask ? mask : ~0ull;
  return KWS_OK;
}

kws_status kws_profile_reset(kws_graph *g) {
  if (!g) return kws::fail(KWS_EINVAL, "null graph");
  std::lock_guard<std::mutex> lk(g->mu);
  g->prof.reset();
  return KWS_OK;
}

kws_status kws_profile_read(kws_graph *g, int32_t id, int64_t *launches, double *total_ms) {
  if (!g || !launches || !total_ms) return kws::fail(KWS_EINVAL, "null argument");
  if (id < 0 || id >= kws::KC_COUNT) return kws::fail(KWS_EINVAL, "no kernel class %d", id);
  std::lock_guard<std::mutex> lk(g->mu);
  *launches = g->prof.launches[id];
  *total_ms = g->prof.total_ms[id];
  return KWS_OK;
}

const char *kws_profile_name(int32_t id) { return kws::kernel_class_name(id); }

kws_status kws_last_batch_stats(kws_graph *g, kws_batch_stats *st) {
  if (!g || !st) return kws::fail(KWS_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g->mu);
  *st = g->last;
  return KWS_OK;
}

}  // extern "C"
