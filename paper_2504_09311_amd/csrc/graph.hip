// Graph store: validation, device copies, reverse CSR, label inverted index
// keyed by type preorder, and the out-degree bins used by the pull kernels.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <thread>

#include "kws_internal.h"

namespace kws {
namespace {

__global__ void k_count_keys(const int32_t *__restrict__ keys, int64_t len, int32_t *__restrict__ cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[keys[i]], 1);
}

// Work-efficient exclusive scan in three launches: per-block totals, one
// block scanning the totals, then per-block scans offset by the totals.
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;

__device__ int32_t block_exclusive_scan(int32_t x, int32_t *total) {
  __shared__ int32_t wsum[BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t incl = x;
  for (int off = 1; off < 64; off <<= 1) {
    int32_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int32_t base = 0, all = 0;
  for (int w = 0; w < BLOCK / 64; w++) {
    if (w < wid) base += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return base + incl - x;
}

__global__ void k_scan_tiles(const int32_t *__restrict__ in, int64_t len, int32_t *__restrict__ tile_sum) {
  int64_t b = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int32_t s = 0;
  for (int i = 0; i < SCAN_ITEMS; i++)
    if (b + i < len) s += in[b + i];
  int32_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int32_t *__restrict__ sums, int64_t count) {
  int32_t carry = 0;
  for (int64_t base = 0; base < count; base += BLOCK) {
    int64_t i = base + threadIdx.x;
    int32_t x = i < count ? sums[i] : 0, tot;
    int32_t ex = block_exclusive_scan(x, &tot);
    if (i < count) sums[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

__global__ void k_scan_apply(const int32_t *__restrict__ in, int64_t len, const int32_t *__restrict__ tile_off,
                             int32_t *__restrict__ out) {
  int64_t b = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS], s = 0;
  for (int i = 0; i < SCAN_ITEMS; i++) {
    v[i] = b + i < len ? in[b + i] : 0;
    s += v[i];
  }
  int32_t tot;
  int32_t ex = block_exclusive_scan(s, &tot) + tile_off[blockIdx.x];
  for (int i = 0; i < SCAN_ITEMS; i++) {
    if (b + i < len) out[b + i] = ex;
    ex += v[i];
  }
}

// out[0..len] = exclusive prefix of in[0..len) with out[len] = total
kws_status exclusive_scan(const int32_t *in, int64_t len, int32_t *out, hipStream_t s) {
  int64_t tiles = (len + SCAN_TILE - 1) / SCAN_TILE;
  int32_t *sums = (int32_t *)dev_alloc(sizeof(int32_t) * (size_t)(tiles + 1));
  if (!sums) return fail(KWS_ENOMEM, "scan scratch");
  if (tiles > 0) {
    k_scan_tiles<<<(unsigned)tiles, BLOCK, 0, s>>>(in, len, sums);
    k_scan_sums<<<1, BLOCK, 0, s>>>(sums, tiles);
    k_scan_apply<<<(unsigned)tiles, BLOCK, 0, s>>>(in, len, sums, out);
  }
  // out[len] = out[len-1] + in[len-1]
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  int32_t last_ex = 0, last_in = 0;
  if (e == hipSuccess && len > 0) e = hipMemcpy(&last_ex, out + len - 1, 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && len > 0) e = hipMemcpy(&last_in, in + len - 1, 4, hipMemcpyDeviceToHost);
  int32_t total = last_ex + last_in;
  if (e == hipSuccess) e = hipMemcpy(out + len, &total, 4, hipMemcpyHostToDevice);
  dev_free(sums);
  if (e != hipSuccess) return fail(KWS_EDEVICE, "scan: %s", hipGetErrorString(e));
  return KWS_OK;
}

// rev_col[cursor[col[e]]++] = source of e; the source is found by binary search
__global__ void k_reverse_scatter(const int32_t *__restrict__ fwd_ptr, const int32_t *__restrict__ fwd_col,
                                  int32_t n, int64_t m, int32_t *__restrict__ cursor,
                                  int32_t *__restrict__ rev_col) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = n;   // largest u with fwd_ptr[u] <= e
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) >> 1;
      if (fwd_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    int32_t pos = atomicAdd(&cursor[fwd_col[e]], 1);
    rev_col[pos] = lo;
  }
}

// keys of the (vertex, label) pairs: preorder key of the label
__global__ void k_label_keys(const int32_t *__restrict__ lab, int64_t len, const int32_t *__restrict__ pre,
                             int32_t *__restrict__ keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = pre[lab[i]];
}

__global__ void k_label_scatter(const int32_t *__restrict__ lab_ptr, int32_t n, const int32_t *__restrict__ keys,
                                int32_t *__restrict__ cursor, int32_t *__restrict__ inv_vtx) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    for (int32_t i = lab_ptr[v]; i < lab_ptr[v + 1]; i++) {
      int32_t pos = atomicAdd(&cursor[keys[i]], 1);
      inv_vtx[pos] = (int32_t)v;
    }
  }
}

unsigned grid_for(int64_t items) {
  int64_t b = (items + BLOCK - 1) / BLOCK;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

template <class T>
kws_status upload(T **dst, const T *src, size_t count, int64_t *bytes, const char *what) {
  *dst = (T *)dev_alloc(sizeof(T) * std::max<size_t>(count, 1));
  if (!*dst) return fail(KWS_ENOMEM, "device allocation for %s (%zu bytes)", what, sizeof(T) * count);
  *bytes += (int64_t)(sizeof(T) * std::max<size_t>(count, 1));
  if (count) KWS_HIP(hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
  return KWS_OK;
}

kws_status alloc_dev(int32_t **dst, size_t count, int64_t *bytes, const char *what) {
  *dst = (int32_t *)dev_alloc(sizeof(int32_t) * std::max<size_t>(count, 1));
  if (!*dst) return fail(KWS_ENOMEM, "device allocation for %s (%zu bytes)", what, 4 * count);
  *bytes += (int64_t)(sizeof(int32_t) * std::max<size_t>(count, 1));
  return KWS_OK;
}

kws_status validate(const kws_graph_desc *d) {
  if (!d) return fail(KWS_EINVAL, "null graph description");
  if (d->n < 1) return fail(KWS_EINVAL, "n must be >= 1 (got %d)", d->n);
  if (d->m < 0) return fail(KWS_EINVAL, "negative m");
  if (d->m >= ((int64_t)1 << 31)) return fail(KWS_EOVERFLOW, "m = %lld does not fit an int32 CSR", (long long)d->m);
  if (!d->row_ptr || (d->m > 0 && !d->col) || !d->lab_ptr)
    return fail(KWS_EINVAL, "missing CSR or label arrays");
  if (d->n_labels < 1) return fail(KWS_EINVAL, "n_labels must be >= 1");
  if (d->row_ptr[0] != 0) return fail(KWS_EINVAL, "row_ptr[0] != 0");
  for (int32_t u = 0; u < d->n; u++)
    if (d->row_ptr[u + 1] < d->row_ptr[u]) return fail(KWS_EINVAL, "row_ptr decreases at %d", u);
  if ((int64_t)d->row_ptr[d->n] != d->m) return fail(KWS_EINVAL, "row_ptr[n] != m");
  for (int64_t e = 0; e < d->m; e++)
    if (d->col[e] < 0 || d->col[e] >= d->n) return fail(KWS_EINVAL, "col[%lld] out of range", (long long)e);
  if (d->lab_ptr[0] != 0) return fail(KWS_EINVAL, "lab_ptr[0] != 0");
  for (int32_t v = 0; v < d->n; v++)
    if (d->lab_ptr[v + 1] < d->lab_ptr[v]) return fail(KWS_EINVAL, "lab_ptr decreases at %d", v);
  int64_t nl = d->lab_ptr[d->n];
  if (nl > 0 && !d->lab) return fail(KWS_EINVAL, "missing lab array");
  for (int64_t i = 0; i < nl; i++)
    if (d->lab[i] < 0 || d->lab[i] >= d->n_labels) return fail(KWS_EINVAL, "lab[%lld] out of range", (long long)i);
  if (d->type_parent)
    for (int32_t t = 0; t < d->n_labels; t++)
      if (d->type_parent[t] < -1 || d->type_parent[t] >= d->n_labels || d->type_parent[t] == t)
        return fail(KWS_EINVAL, "type_parent[%d] invalid", t);
  return KWS_OK;
}

// Preorder numbering of the type forest: roots and children in ascending id
// order. pre[t] is t's position; t and its descendants occupy
// [pre[t], pre[t] + span[t]). Fails if the parents contain a cycle.
kws_status type_preorder(const int32_t *parent, int32_t nt, std::vector<int32_t> &pre,
                         std::vector<int32_t> &span, int32_t *depth) {
  *depth = 0;
  pre.assign(nt, -1);
  span.assign(nt, 1);
  if (!parent) {
    std::iota(pre.begin(), pre.end(), 0);
    return KWS_OK;
  }
  std::vector<int32_t> cptr(nt + 1, 0), kids(nt);
  for (int32_t t = 0; t < nt; t++)
    if (parent[t] >= 0) cptr[parent[t] + 1]++;
  for (int32_t t = 0; t < nt; t++) cptr[t + 1] += cptr[t];
  std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
  for (int32_t t = 0; t < nt; t++)
    if (parent[t] >= 0) kids[fill[parent[t]]++] = t;   // ascending t per parent
  int32_t next = 0;
  std::vector<std::pair<int32_t, int32_t>> stack;     // (type, next child index)
  for (int32_t r = 0; r < nt; r++) {
    if (parent[r] >= 0) continue;
    pre[r] = next++;
    stack.push_back({r, cptr[r]});
    while (!stack.empty()) {
      auto &top = stack.back();
      if (top.second < cptr[top.first + 1]) {
        int32_t c = kids[top.second++];
        pre[c] = next++;
        stack.push_back({c, cptr[c]});
        *depth = std::max(*depth, (int32_t)stack.size() - 1);
      } else {
        span[top.first] = next - pre[top.first];
        stack.pop_back();
      }
    }
  }
  if (next != nt) return fail(KWS_EINVAL, "type_parent contains a cycle");
  return KWS_OK;
}

// Rows of the forward CSR sorted by neighbour id (the answer walk stops at
// the first qualifying neighbour). Returns an empty vector when the input is
// already sorted.
std::vector<int32_t> sorted_rows(const int32_t *row_ptr, const int32_t *col, int32_t n, int64_t m) {
  bool sorted = true;
  for (int32_t u = 0; u < n && sorted; u++)
    for (int32_t e = row_ptr[u] + 1; e < row_ptr[u + 1]; e++)
      if (col[e - 1] > col[e]) { sorted = false; break; }
  std::vector<int32_t> out;
  if (sorted) return out;
  out.assign(col, col + m);
  const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int t = 0; t < nt; t++)
    th.emplace_back([&, t] {
      for (int32_t u = t; u < n; u += nt) std::sort(out.begin() + row_ptr[u], out.begin() + row_ptr[u + 1]);
    });
  for (auto &x : th) x.join();
  return out;
}

}  // namespace

kws_status load_graph(const kws_graph_desc *d, kws_graph **out) {
  if (!out) return fail(KWS_EINVAL, "null output handle");
  *out = nullptr;
  KWS_TRY(validate(d));
  std::vector<int32_t> pre, span;
  int32_t depth = 0;
  KWS_TRY(type_preorder(d->type_parent, d->n_labels, pre, span, &depth));

  kws_graph *g = new kws_graph();
  // load-time scratch; a failure anywhere frees it with the graph
  int32_t *cnt = nullptr, *d_pre = nullptr, *keys = nullptr, *icnt = nullptr;
  auto free_scratch = [&]() {
    for (int32_t **p : {&cnt, &d_pre, &keys, &icnt}) {
      dev_free(*p);
      *p = nullptr;
    }
  };
  auto bail = [&](kws_status st) {
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    free_scratch();
    free_graph(g);
    return st;
  };
  KWS_HIP(hipGetDevice(&g->device));
  g->n = d->n;
  g->m = d->m;
  g->n_labels = d->n_labels;
  g->h_lab_total = d->lab_ptr[d->n];
  g->type_depth = depth;
  g->hier = d->type_parent != nullptr;
  g->pre = pre;
  g->span = span;
  default_options(&g->opt);
  if (hipStreamCreateWithFlags(&g->own_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(KWS_EDEVICE, "stream creation failed"));
  g->stream = g->own_stream;
  hipStream_t s = g->stream;
  const int32_t n = d->n;
  const int64_t m = d->m, nl = d->lab_ptr[n];
  int64_t bytes = 0;
  kws_status st;
#define STEP(x) do { st = (x); if (st != KWS_OK) return bail(st); } while (0)
#define HSTEP(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return bail(fail(KWS_EDEVICE, "%s: %s", #x, hipGetErrorString(e_))); } while (0)

  // forward CSR, rows sorted by neighbour id
  STEP(upload(&g->fwd_ptr, d->row_ptr, (size_t)n + 1, &bytes, "row_ptr"));
  {
    std::vector<int32_t> sc = sorted_rows(d->row_ptr, d->col, n, m);
    STEP(upload(&g->fwd_col, sc.empty() ? d->col : sc.data(), (size_t)m, &bytes, "col"));
  }
  // reverse CSR: in-degree count, scan, scatter
  int32_t *cursor = nullptr;
  int64_t scratch = 0;
  STEP(alloc_dev(&cnt, (size_t)n + 1, &scratch, "in-degree"));
  STEP(alloc_dev(&g->rev_ptr, (size_t)n + 1, &bytes, "rev_ptr"));
  STEP(alloc_dev(&g->rev_col, (size_t)m, &bytes, "rev_col"));
  HSTEP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * ((size_t)n + 1), s));
  if (m > 0) k_count_keys<<<grid_for(m), BLOCK, 0, s>>>(g->fwd_col, m, cnt);
  HSTEP(hipGetLastError());
  STEP(exclusive_scan(cnt, n, g->rev_ptr, s));
  HSTEP(hipMemcpyAsync(cnt, g->rev_ptr, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
  cursor = cnt;
  if (m > 0) k_reverse_scatter<<<grid_for(m), BLOCK, 0, s>>>(g->fwd_ptr, g->fwd_col, n, m, cursor, g->rev_col);
  HSTEP(hipGetLastError());
  HSTEP(hipStreamSynchronize(s));
  dev_free(cnt);
  cnt = nullptr;

  // inverted index over preorder keys
  STEP(upload(&g->lab_ptr, d->lab_ptr, (size_t)n + 1, &bytes, "lab_ptr"));
  STEP(upload(&g->lab, d->lab, (size_t)nl, &bytes, "lab"));
  int32_t *d_lab_ptr = g->lab_ptr, *d_lab = g->lab;
  if (d->type_parent) STEP(upload(&g->tparent, d->type_parent, (size_t)g->n_labels, &bytes, "type parents"));
  STEP(upload(&d_pre, pre.data(), pre.size(), &scratch, "type preorder"));
  STEP(alloc_dev(&keys, (size_t)nl, &scratch, "label keys"));
  STEP(alloc_dev(&icnt, (size_t)g->n_labels + 1, &scratch, "label counts"));
  STEP(alloc_dev(&g->inv_ptr, (size_t)g->n_labels + 1, &bytes, "inv_ptr"));
  STEP(alloc_dev(&g->inv_vtx, (size_t)nl, &bytes, "inv_vtx"));
  HSTEP(hipMemsetAsync(icnt, 0, sizeof(int32_t) * ((size_t)g->n_labels + 1), s));
  if (nl > 0) {
    k_label_keys<<<grid_for(nl), BLOCK, 0, s>>>(d_lab, nl, d_pre, keys);
    k_count_keys<<<grid_for(nl), BLOCK, 0, s>>>(keys, nl, icnt);
  }
  HSTEP(hipGetLastError());
  STEP(exclusive_scan(icnt, g->n_labels, g->inv_ptr, s));
  HSTEP(hipMemcpyAsync(icnt, g->inv_ptr, sizeof(int32_t) * (size_t)g->n_labels, hipMemcpyDeviceToDevice, s));
  if (nl > 0) k_label_scatter<<<grid_for(n), BLOCK, 0, s>>>(d_lab_ptr, n, keys, icnt, g->inv_vtx);
  HSTEP(hipGetLastError());
  g->h_inv_ptr.resize((size_t)g->n_labels + 1);
  HSTEP(hipMemcpyAsync(g->h_inv_ptr.data(), g->inv_ptr, sizeof(int32_t) * ((size_t)g->n_labels + 1),
                       hipMemcpyDeviceToHost, s));
  HSTEP(hipStreamSynchronize(s));
  free_scratch();

  // degree facts and pull bins (host side: the CSR is already here)
  std::vector<int32_t> indeg(n, 0);
  for (int64_t e = 0; e < m; e++) indeg[d->col[e]]++;
  std::vector<int32_t> bins[BIN_COUNT];
  std::vector<int32_t> hv, hb, he, hubs, zeros;
  for (int32_t u = 0; u < n; u++) {
    int32_t b = d->row_ptr[u], e = d->row_ptr[u + 1], deg = e - b;
    g->max_out = std::max(g->max_out, deg);
    g->max_in = std::max(g->max_in, indeg[u]);
    if (deg == 0) {
      zeros.push_back(u);
      continue;
    }
    if (deg <= BIN_SMALL_MAX) bins[BIN_SMALL].push_back(u);
    else if (deg <= BIN_MEDIUM_MAX) bins[BIN_MEDIUM].push_back(u);
    else if (deg <= BIN_LARGE_MAX) bins[BIN_LARGE].push_back(u);
    else {
      hubs.push_back(u);
      for (int32_t c = b; c < e; c += HUB_CHUNK) {
        hv.push_back(u); hb.push_back(c); he.push_back(std::min(e, c + HUB_CHUNK));
      }
    }
  }
  std::vector<int32_t> all;
  for (int b = 0; b < BIN_COUNT; b++) {
    // longest rows first inside a bin, ties by vertex id
    std::stable_sort(bins[b].begin(), bins[b].end(), [&](int32_t x, int32_t y) {
      return d->row_ptr[x + 1] - d->row_ptr[x] > d->row_ptr[y + 1] - d->row_ptr[y];
    });
    g->bin_begin[b] = (int64_t)all.size();
    all.insert(all.end(), bins[b].begin(), bins[b].end());
  }
  g->bin_begin[BIN_COUNT] = (int64_t)all.size();
  g->n_hub = (int64_t)hv.size();
  STEP(upload(&g->bin_vtx, all.data(), all.size(), &bytes, "pull bins"));
  STEP(upload(&g->hub_v, hv.data(), hv.size(), &bytes, "hub chunks"));
  STEP(upload(&g->hub_b, hb.data(), hb.size(), &bytes, "hub chunks"));
  STEP(upload(&g->hub_e, he.data(), he.size(), &bytes, "hub chunks"));
  g->n_hubv = (int64_t)hubs.size();
  g->n_zero = (int64_t)zeros.size();
  STEP(upload(&g->hub_vtx, hubs.data(), hubs.size(), &bytes, "hub vertices"));
  STEP(upload(&g->zero_vtx, zeros.data(), zeros.size(), &bytes, "vertices without out-edges"));
  g->device_bytes = bytes;
#undef STEP
#undef HSTEP
  *out = g;
  return KWS_OK;
}

void free_graph(kws_graph *g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  drop_pending(g);
  for (auto &e : g->graphs)
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
  g->graphs.clear();
  g->eng.release();
  g->prof.release();
  int32_t *ptrs[] = {g->fwd_ptr, g->fwd_col, g->rev_ptr, g->rev_col, g->inv_ptr, g->inv_vtx,
                     g->lab_ptr, g->lab, g->tparent, g->bin_vtx, g->hub_v, g->hub_b, g->hub_e,
                     g->hub_vtx, g->zero_vtx};
  for (int32_t *p : ptrs) dev_free(p);
  if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
  delete g;
}

}  // namespace kws
