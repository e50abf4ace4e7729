// autotune.hip -- picks delta (bucket width), the partition count P, the
// lag window and the workgroup size for sssp_solve by timing settings on the
// device, one coordinate at a time from the library's own defaults (delta
// over multiples of the mean arc cost sampled from the device and one
// unbounded bucket; then P around its default; then lag; then the workgroup
// size; then the grid size).  Each setting is timed from five sources and
// scored by the median time; a setting replaces the best so far only when
// its median is more than 3% faster and it is not slower from the caller's
// own source.
//
// The bucket width trades the two effects the paper's related-work section
// describes for delta-stepping: a wide bucket exposes more parallel work per
// round but re-relaxes more vertices, a narrow one needs more rounds.
// Results are cached per device and coarse graph signature in the process and
// can be persisted as JSON; solves with automatic options consult the cache.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace sssp_impl {

namespace {
std::mutex g_mu;
std::map<std::string, sssp_opts> g_cache;

// "<arch>/<CUs>" of the current device (queried once per device).
std::string device_tag() {
  static std::map<int, std::string> tags;  // guarded by g_mu
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  auto it = tags.find(dev);
  if (it != tags.end()) return it->second;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  return tags[dev] = arch + "/" + std::to_string(prop.multiProcessorCount);
}

// Coarse signature: graphs of the same weight type, the same ceil(log2 n)
// and the same floor(log2) of the average degree share an entry.
std::string graph_key(const sssp_csr &g) {
  int ln = 0;
  while ((1ll << ln) < (long long)g.n) ln++;
  const double avg = g.m > 0 ? (double)g.m / g.n : 0.0;
  const int ld = avg > 0 ? (int)std::floor(std::log2(avg)) : -99;
  return device_tag() + "|w=" + std::to_string(g.wtype) + "|log2n=" + std::to_string(ln) +
         "|log2deg=" + std::to_string(ld);
}

// Batch signature: weight type, number of graphs and of solves, ceil(log2)
// of the total vertex count and floor(log2) of the average degree.
std::string batch_key(int num_graphs, const sssp_csr *graphs, int num_solves) {
  long long n = 0, m = 0;
  for (int i = 0; i < num_graphs; i++) {
    n += graphs[i].n;
    m += graphs[i].m;
  }
  int ln = 0;
  while ((1ll << ln) < n) ln++;
  const double avg = m > 0 ? (double)m / (double)n : 0.0;
  const int ld = avg > 0 ? (int)std::floor(std::log2(avg)) : -99;
  return device_tag() + "|batch|w=" + std::to_string(graphs[0].wtype) + "|g=" +
         std::to_string(num_graphs) + "|s=" + std::to_string(num_solves) + "|log2n=" +
         std::to_string(ln) + "|log2deg=" + std::to_string(ld);
}

void load_json(const char *path) {
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
  std::fclose(f);
  // one entry per line: {"key": "...", "delta": D, "num_partitions": P,
  //                      "wg_size": W, "num_workgroups": G, "lag": L}
  size_t pos = 0;
  while ((pos = text.find("{\"key\": \"", pos)) != std::string::npos) {
    const size_t ks = pos + 9;
    const size_t ke = text.find('"', ks);
    if (ke == std::string::npos) break;
    const std::string key = text.substr(ks, ke - ks);
    double delta = 0;
    int P = 0, W = 0, G = 0, Lg = 0;
    if (std::sscanf(text.c_str() + ke + 1,
                    ", \"delta\": %lf, \"num_partitions\": %d, \"wg_size\": %d, "
                    "\"num_workgroups\": %d, \"lag\": %d",
                    &delta, &P, &W, &G, &Lg) == 5) {
      sssp_opts o;
      std::memset(&o, 0, sizeof(o));
      o.delta = delta;
      o.num_partitions = P;
      o.wg_size = W;
      o.num_workgroups = G;
      o.lag = Lg;
      g_cache[key] = o;
    }
    pos = ke;
  }
}

void save_json(const char *path) {
  FILE *f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "[\n");
  size_t i = 0;
  for (const auto &kv : g_cache) {
    const sssp_opts &o = kv.second;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"delta\": %.17g, \"num_partitions\": %d, \"wg_size\": %d, "
                 "\"num_workgroups\": %d, \"lag\": %d}%s\n",
                 kv.first.c_str(), o.delta, o.num_partitions, o.wg_size, o.num_workgroups,
                 o.lag, ++i < g_cache.size() ? "," : "");
  }
  std::fprintf(f, "]\n");
  std::fclose(f);
}

}  // namespace

bool autotune_lookup(const sssp_csr &g, sssp_opts *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_cache.empty()) return false;
  auto it = g_cache.find(graph_key(g));
  if (it == g_cache.end()) return false;
  *out = it->second;
  return true;
}

bool autotune_lookup_batch(int num_graphs, const sssp_csr *graphs, int num_solves,
                           sssp_opts *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_cache.empty()) return false;
  auto it = g_cache.find(batch_key(num_graphs, graphs, num_solves));
  if (it == g_cache.end()) return false;
  *out = it->second;
  return true;
}

}  // namespace sssp_impl

using namespace sssp_impl;

extern "C" int sssp_autotune(const sssp_csr *g, int32_t source, void *dist_scratch,
                             sssp_opts *best, const char *cache_path, void *ws,
                             size_t *ws_bytes, void *stream) {
  int rc = check_csr(g);
  if (rc) return rc;
  if (!ws_bytes || !best) return SSSP_ERR_ARG;
  if (source < 0 || source >= g->n) return SSSP_ERR_SOURCE;
  // workspace: the largest requirement over the candidate partition counts
  size_t need = 0;
  {
    const int p0 = best->num_partitions > 0 ? best->num_partitions : default_parts(g->n, g->m);
    for (long long p : {(long long)p0 / 4, (long long)p0, (long long)p0 * 4}) {
      sssp_opts o;
      sssp_opts_init(&o);
      o.num_partitions = (int)std::max(1ll, std::min(p, (long long)g->n));
      o.flags = SSSP_F_NO_AUTOTUNE;
      size_t b = 0;
      if ((rc = sssp_solve(g, source, &o, nullptr, nullptr, nullptr, nullptr, nullptr, &b,
                           stream)))
        return rc;
      need = std::max(need, b);
    }
  }
  if (!ws) {
    *ws_bytes = need;
    return SSSP_OK;
  }
  if (!dist_scratch) return SSSP_ERR_ARG;
  if ((rc = check_ws(ws, *ws_bytes, need))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  sssp_opts sy;
  sssp_opts_init(&sy);
  sy.flags = SSSP_F_SYNC;
  if ((rc = check_sync(sy, st))) return rc;
  if (cache_path) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_json(cache_path);
  }

  // mean arc cost from a sample of the weights
  double mean_w = g->wtype == SSSP_W_U32 ? 128.0 : 1.0;
  if (g->m > 0) {
    const int k = std::min(g->m, 1 << 16);
    std::vector<uint32_t> h(k);
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(h.data(), g->w, sizeof(uint32_t) * k, hipMemcpyDeviceToHost) != hipSuccess)
      return SSSP_ERR_HIP;
    double s = 0;
    for (uint32_t x : h) {
      float f;
      std::memcpy(&f, &x, 4);
      s += g->wtype == SSSP_W_U32 ? (double)x : (double)f;
    }
    mean_w = std::max(s / k, g->wtype == SSSP_W_U32 ? 1.0 : 1e-30);
  }

  // Sources timed for every candidate: the caller's, and four more vertices
  // with out-arcs at fixed quantiles of the id range (the cache entry serves
  // every source of graphs with this signature, so one source's timing is a
  // poor guide).  A candidate's score is the median of its per-source times.
  std::vector<int32_t> sources{source};
  {
    std::vector<int32_t> rp(g->n + 1);
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(rp.data(), g->row_ptr, sizeof(int32_t) * (g->n + 1), hipMemcpyDeviceToHost) !=
            hipSuccess)
      return SSSP_ERR_HIP;
    for (double q : {0.2, 0.4, 0.6, 0.8}) {
      int v = (int)(q * (g->n - 1));
      for (int k = 0; k < g->n && rp[v + 1] == rp[v]; k++) v = (v + 1) % g->n;
      if (rp[v + 1] > rp[v] && v != source) sources.push_back(v);
    }
  }
  const int ns = (int)sources.size();

  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return SSSP_ERR_HIP;
  struct Cleanup {
    hipEvent_t a, b;
    ~Cleanup() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      g_solve_time_limit_s = 30.0;
    }
  } cleanup{e0, e1};
  const sssp_opts fixed = *best;
  // Start from exactly what sssp_solve does with automatic options (delta 0
  // = the width computed on the device, the default P, workgroup size, grid
  // and lag), so the defaults are always a candidate and the tuned choice
  // never scores worse than them.
  const bool dense = g->m >= 8ll * g->n;
  sssp_opts cur;  // the best so far; fields fixed by the caller never change
  sssp_opts_init(&cur);
  cur.delta = fixed.delta;
  cur.num_partitions = fixed.num_partitions > 0 ? fixed.num_partitions
                                                : default_parts(g->n, g->m);
  cur.wg_size = fixed.wg_size ? fixed.wg_size : (dense ? 512 : 256);
  cur.lag = fixed.lag;
  cur.num_workgroups = fixed.num_workgroups;
  float best_score = 1e30f;
  std::vector<float> best_per(ns, 1e30f);
  bool found = false;
  // Times one setting from every source (best of two runs each).  Each run
  // is cut short by the device time limit at 4x that source's time under
  // the best setting so far; a setting cut short is skipped.
  auto trial = [&](const sssp_opts &cand) -> int {
    sssp_opts o = cand;
    o.flags = SSSP_F_NO_AUTOTUNE | SSSP_F_SYNC;
    o.event_start = e0;
    o.event_stop = e1;
    std::vector<float> per(ns, 1e30f);
    for (int si = 0; si < ns; si++) {
      g_solve_time_limit_s = found ? std::min(30.0, std::max(0.02, 4e-3 * best_per[si])) : 30.0;
      for (int rep = 0; rep < 2; rep++) {
        size_t b = *ws_bytes;
        const int r = sssp_solve(g, sources[si], &o, dist_scratch, nullptr, nullptr, nullptr, ws,
                                 &b, stream);
        if (r == SSSP_ERR_TIMEOUT && found) return SSSP_OK;
        if (r != SSSP_OK) return r;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return SSSP_ERR_HIP;
        per[si] = std::min(per[si], ms);
      }
    }
    std::vector<float> sorted = per;
    std::sort(sorted.begin(), sorted.end());
    const float score = sorted[ns / 2];
    // a new setting must win the median by more than run-to-run noise (3%)
    // and must not be slower from the caller's own source: the defaults,
    // tried first, stay unless something is clearly faster
    if (!found || (score < 0.97f * best_score && per[0] <= best_per[0])) {
      best_score = score;
      best_per = per;
      cur = cand;
      found = true;
    }
    return SSSP_OK;
  };
  // coordinate descent: bucket width, then partitions, lag, workgroup size
  if ((rc = trial(cur))) return rc;
  if (fixed.delta == 0) {
    const sssp_opts base = cur;
    for (double f : {0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0, -1.0}) {
      sssp_opts c = base;
      c.delta = f < 0 ? -1.0 : mean_w * f;
      if ((rc = trial(c))) return rc;
    }
  }
  if (fixed.num_partitions == 0) {
    const sssp_opts base = cur;
    for (int k : {-2, -1, 1, 2}) {
      sssp_opts c = base;
      const long long p = k < 0 ? base.num_partitions >> -k : (long long)base.num_partitions << k;
      c.num_partitions = (int)std::max(1ll, std::min(p, (long long)g->n));
      if (c.num_partitions == base.num_partitions) continue;
      if ((rc = trial(c))) return rc;
    }
  }
  if (fixed.lag == 0 && cur.delta >= 0) {  // the lag window needs a finite bucket width
    const sssp_opts base = cur;
    for (int l : {2, 4, -1}) {
      sssp_opts c = base;
      c.lag = l;
      if ((rc = trial(c))) return rc;
    }
  }
  if (fixed.wg_size == 0) {
    sssp_opts c = cur;
    c.wg_size = cur.wg_size == 512 ? 256 : 512;
    if ((rc = trial(c))) return rc;
  }
  if (fixed.num_workgroups == 0) {
    const sssp_opts base = cur;
    const int cus = device_info().cus;
    for (int gw : {cus / 2, cus, 2 * cus}) {
      sssp_opts c = base;
      c.num_workgroups = gw;
      if ((rc = trial(c))) return rc;
    }
  }
  if (!found) return SSSP_ERR_TIMEOUT;
  sssp_opts best_o = cur;
  best_o.flags = 0;
  best_o.event_start = nullptr;
  best_o.event_stop = nullptr;
  *best = best_o;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[graph_key(*g)] = best_o;
    if (cache_path) save_json(cache_path);
  }
  return SSSP_OK;
}

extern "C" int sssp_autotune_batch(int32_t num_graphs, const sssp_csr *graphs, int32_t num_solves,
                                   const int32_t *solve_graph, const int32_t *solve_source,
                                   const int64_t *out_offset, void *dist_scratch,
                                   sssp_opts *best, const char *cache_path, void *ws,
                                   size_t *ws_bytes, void *stream) {
  if (!ws_bytes || !best || num_graphs < 1 || !graphs) return SSSP_ERR_ARG;
  const sssp_opts fixed = *best;
  // candidate partition counts (0 = each graph's default)
  std::vector<int> parts;
  if (fixed.num_partitions > 0) parts = {fixed.num_partitions};
  else parts = {0, 4, 16, 64};
  int rc;
  size_t need = 0;
  for (int p : parts) {
    sssp_opts o;
    sssp_opts_init(&o);
    o.num_partitions = p;
    o.flags = SSSP_F_NO_AUTOTUNE;
    size_t b = 0;
    if ((rc = sssp_solve_batch(num_graphs, graphs, num_solves, solve_graph, solve_source,
                               out_offset, &o, nullptr, nullptr, nullptr, nullptr, nullptr, &b,
                               stream)))
      return rc;
    need = std::max(need, b);
  }
  if (!ws) {
    *ws_bytes = need;
    return SSSP_OK;
  }
  if (!dist_scratch) return SSSP_ERR_ARG;
  if ((rc = check_ws(ws, *ws_bytes, need))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  sssp_opts sy;
  sssp_opts_init(&sy);
  sy.flags = SSSP_F_SYNC;
  if ((rc = check_sync(sy, st))) return rc;
  if (cache_path) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_json(cache_path);
  }
  // mean arc cost from a sample of the first graph's weights
  double mean_w = graphs[0].wtype == SSSP_W_U32 ? 128.0 : 1.0;
  if (graphs[0].m > 0) {
    const int k = std::min(graphs[0].m, 1 << 16);
    std::vector<uint32_t> h(k);
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(h.data(), graphs[0].w, sizeof(uint32_t) * k, hipMemcpyDeviceToHost) !=
            hipSuccess)
      return SSSP_ERR_HIP;
    double sum = 0;
    for (uint32_t x : h) {
      float f;
      std::memcpy(&f, &x, 4);
      sum += graphs[0].wtype == SSSP_W_U32 ? (double)x : (double)f;
    }
    mean_w = std::max(sum / k, graphs[0].wtype == SSSP_W_U32 ? 1.0 : 1e-30);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return SSSP_ERR_HIP;
  struct Cleanup {
    hipEvent_t a, b;
    ~Cleanup() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      g_solve_time_limit_s = 30.0;
    }
  } cleanup{e0, e1};
  sssp_opts cur;
  sssp_opts_init(&cur);
  cur.delta = fixed.delta;  // 0 = each graph's automatic width
  cur.num_partitions = fixed.num_partitions;
  cur.wg_size = fixed.wg_size ? fixed.wg_size : 512;
  cur.num_workgroups = fixed.num_workgroups;
  float best_ms = 1e30f;
  bool found = false;
  auto trial = [&](const sssp_opts &cand) -> int {
    g_solve_time_limit_s = found ? std::min(30.0, std::max(0.02, 4e-3 * best_ms)) : 30.0;
    sssp_opts o = cand;
    o.flags = SSSP_F_NO_AUTOTUNE | SSSP_F_SYNC;
    o.event_start = e0;
    o.event_stop = e1;
    float ms_min = 1e30f;
    for (int rep = 0; rep < 2; rep++) {
      size_t b = *ws_bytes;
      const int r = sssp_solve_batch(num_graphs, graphs, num_solves, solve_graph, solve_source,
                                     out_offset, &o, dist_scratch, nullptr, nullptr, nullptr,
                                     ws, &b, stream);
      if (r == SSSP_ERR_TIMEOUT && found) return SSSP_OK;
      if (r != SSSP_OK) return r;
      float ms = 0;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return SSSP_ERR_HIP;
      ms_min = std::min(ms_min, ms);
    }
    if (ms_min < best_ms) {
      best_ms = ms_min;
      cur = cand;
      found = true;
    }
    return SSSP_OK;
  };
  if ((rc = trial(cur))) return rc;
  if (fixed.delta == 0) {
    const sssp_opts base = cur;
    for (double f : {0.25, 0.5, 1.0, 2.0, 4.0}) {
      sssp_opts c = base;
      c.delta = mean_w * f;
      if ((rc = trial(c))) return rc;
    }
  }
  if (fixed.num_partitions == 0) {
    const sssp_opts base = cur;
    for (int p : parts) {
      if (p == base.num_partitions) continue;
      sssp_opts c = base;
      c.num_partitions = p;
      if ((rc = trial(c))) return rc;
    }
  }
  if (fixed.wg_size == 0) {
    sssp_opts c = cur;
    c.wg_size = 256;
    if ((rc = trial(c))) return rc;
  }
  if (fixed.num_workgroups == 0) {
    const sssp_opts base = cur;
    const int cus = device_info().cus;
    for (int gw : {cus / 2, 2 * cus, 4 * cus}) {
      sssp_opts c = base;
      c.num_workgroups = gw;
      if ((rc = trial(c))) return rc;
    }
  }
  if (!found) return SSSP_ERR_TIMEOUT;
  sssp_opts out = cur;
  out.flags = 0;
  out.event_start = nullptr;
  out.event_stop = nullptr;
  *best = out;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[batch_key(num_graphs, graphs, num_solves)] = out;
    if (cache_path) save_json(cache_path);
  }
  return SSSP_OK;
}
