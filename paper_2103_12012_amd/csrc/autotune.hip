// autotune.hip -- picks delta (bucket width), the partition count P and the
// workgroup shape for sssp_solve by timing candidates on the device.
//
// The bucket width trades the two effects the paper's related-work section
// describes for delta-stepping: a wide bucket exposes more parallel work per
// round but re-relaxes more vertices, a narrow one needs more rounds.  The
// candidates are multiples of the mean arc cost (sampled from the device).
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

struct Candidate {
  double delta;
  int parts, wg, lag;
};

// Candidates around the defaults; fields the caller fixed in *best are kept.
std::vector<Candidate> candidates(const sssp_csr &g, double mean_w, const sssp_opts &fixed) {
  std::vector<double> deltas;
  if (fixed.delta != 0) {
    deltas.push_back(fixed.delta);
  } else {
    for (double f : {0.25, 0.5, 1.0, 2.0, 8.0, 32.0}) deltas.push_back(mean_w * f);
    deltas.push_back(-1.0);  // one unbounded bucket: asynchronous Bellman-Ford
  }
  std::vector<int> parts;
  if (fixed.num_partitions > 0) {
    parts.push_back(fixed.num_partitions);
  } else {
    const int p0 = default_parts(g.n);
    for (int p : {p0 / 4, p0, p0 * 4}) {
      int q = std::max(1, std::min(p, g.n));
      if (std::find(parts.begin(), parts.end(), q) == parts.end()) parts.push_back(q);
    }
  }
  std::vector<int> wgs;
  if (fixed.wg_size) wgs.push_back(fixed.wg_size);
  else wgs = {256, 512};
  std::vector<int> lags;
  if (fixed.lag) lags.push_back(fixed.lag);
  else lags = {1, 2, -1};
  std::vector<Candidate> out;
  for (double d : deltas)
    for (int p : parts)
      for (int w : wgs)
        for (int l : lags) {
          if (d < 0 && l != lags[0]) continue;  // no window without buckets
          out.push_back({d, p, w, l});
        }
  return out;
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
    const int p0 = best->num_partitions > 0 ? best->num_partitions : default_parts(g->n);
    for (int p : {p0 / 4, p0, p0 * 4}) {
      sssp_opts o;
      sssp_opts_init(&o);
      o.num_partitions = std::max(1, std::min(p, g->n));
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

  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return SSSP_ERR_HIP;
  float best_ms = 1e30f;
  sssp_opts best_o;
  sssp_opts_init(&best_o);
  bool found = false;
  const sssp_opts fixed = *best;
  struct LimitGuard {
    ~LimitGuard() { g_solve_time_limit_s = 30.0; }
  } guard;
  for (const Candidate &c : candidates(*g, mean_w, fixed)) {
    // a candidate slower than 4x the best so far stops at the time limit
    g_solve_time_limit_s = found ? std::min(30.0, std::max(0.02, 4e-3 * best_ms)) : 30.0;
    sssp_opts o;
    sssp_opts_init(&o);
    o.delta = c.delta;
    o.num_partitions = c.parts;
    o.wg_size = c.wg;
    o.lag = c.lag;
    o.num_workgroups = fixed.num_workgroups;
    o.flags = SSSP_F_NO_AUTOTUNE;
    o.event_start = e0;
    o.event_stop = e1;
    float ms_min = 1e30f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; rep++) {
      size_t b = *ws_bytes;
      o.flags = SSSP_F_NO_AUTOTUNE | SSSP_F_SYNC;
      rc = sssp_solve(g, source, &o, dist_scratch, nullptr, nullptr, nullptr, ws, &b, stream);
      if (rc == SSSP_ERR_TIMEOUT && found) {  // slower than the best: skip it
        rc = SSSP_OK;
        ok = false;
        break;
      }
      if (rc != SSSP_OK) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return rc;
      }
      float ms = 0;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        ok = false;
        break;
      }
      ms_min = std::min(ms_min, ms);
    }
    if (ok && ms_min < best_ms) {
      best_ms = ms_min;
      best_o = o;
      found = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!found) return SSSP_ERR_TIMEOUT;
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
