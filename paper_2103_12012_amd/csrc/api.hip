// api.hip -- host side of the C ABI declared in include/sssp.h: argument
// checks, parameter planning, workspace carving and the launch sequence.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"
#include "plan.hpp"

using namespace sssp_impl;

namespace sssp_impl {

const char *strerror_impl(int code) {
  switch (code) {
    case SSSP_OK: return "ok";
    case SSSP_ERR_ARG: return "invalid argument";
    case SSSP_ERR_SOURCE: return "source outside [0, n)";
    case SSSP_ERR_CSR: return "malformed CSR (row_ptr or col)";
    case SSSP_ERR_UNSORTED: return "a CSR row is not sorted by column";
    case SSSP_ERR_WEIGHT: return "invalid fp32 weight (negative, -0.0, NaN or inf)";
    case SSSP_ERR_ZERO_WEIGHT: return "zero weight (backward needs w > 0)";
    case SSSP_ERR_OVERFLOW: return "path length overflow";
    case SSSP_ERR_TIMEOUT: return "max_rounds or time limit reached";
    case SSSP_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case SSSP_ERR_HIP: return "HIP runtime error";
    case SSSP_ERR_CAPTURE: return "SSSP_F_SYNC on a capturing stream";
    case SSSP_ERR_CYCLE: return "predecessor graph has a cycle";
    case SSSP_ERR_TOO_LARGE: return "graph too large for the library's fixed solve workspace";
    default: return "unknown error";
  }
}

// ---------------------------------------------------------------- device info
DevInfo device_info() {
  static std::mutex mu;
  static std::vector<DevInfo> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DevInfo{};
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1);
  if (cache[dev].cus == 0) {
    int cus = 0, khz = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
      khz = 0;
    cache[dev].cus = cus > 0 ? cus : 256;
    cache[dev].wall_khz = khz > 0 ? khz : 100000;
  }
  return cache[dev];
}

// ---------------------------------------------------------------- checks
int check_csr(const sssp_csr *g) {
  if (!g) return SSSP_ERR_ARG;
  // 32-bit vertex and arc indices: n and m leave room for 2n and for the
  // kernels' grid-stride steps (below 2^24) without overflowing an int
  if (g->n < 1 || g->n > SSSP_N_MAX || g->m < 0 || g->m > SSSP_M_MAX) return SSSP_ERR_ARG;
  if (!g->row_ptr) return SSSP_ERR_ARG;
  if (g->m > 0 && (!g->col || !g->w)) return SSSP_ERR_ARG;
  if (g->wtype != SSSP_W_U32 && g->wtype != SSSP_W_F32) return SSSP_ERR_ARG;
  if (g->reserved != 0) return SSSP_ERR_ARG;
  return SSSP_OK;
}

int check_opts(const sssp_opts *o) {
  if (o->wg_size != 0 && o->wg_size != 256 && o->wg_size != 512 && o->wg_size != 1024)
    return SSSP_ERR_ARG;
  if (o->num_partitions < 0 || o->num_workgroups < 0 || o->max_rounds < 0) return SSSP_ERR_ARG;
  if (std::isnan(o->delta)) return SSSP_ERR_ARG;
  const int modes = ((o->flags & SSSP_F_LOCAL_HEAP) != 0) + ((o->flags & SSSP_F_BUFFER_CROSS) != 0) +
                    ((o->flags & SSSP_F_IDLE_PRUNE) != 0);
  if (modes > 1) return SSSP_ERR_ARG;
  return SSSP_OK;
}

int check_ws(void *ws, size_t have, size_t need) {
  if (!ws || have < need || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return SSSP_ERR_WORKSPACE;
  return SSSP_OK;
}

int check_sync(const sssp_opts &o, hipStream_t st) {
  if (!(o.flags & SSSP_F_SYNC)) return SSSP_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return SSSP_ERR_HIP;
  return cs == hipStreamCaptureStatusNone ? SSSP_OK : SSSP_ERR_CAPTURE;
}

// Waits for the stream and returns the device status word.
int finish_sync(const int32_t *dev_status, hipStream_t st) {
  if (hipStreamSynchronize(st) != hipSuccess) return SSSP_ERR_HIP;
  int32_t s = 0;
  if (hipMemcpy(&s, dev_status, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess)
    return SSSP_ERR_HIP;
  return s;
}

// ---------------------------------------------------------------- planning
unsigned long long delta_units(double delta, int wtype) {
  if (delta < 0 || std::isinf(delta)) return DELTA_INF;
  if (wtype == SSSP_W_U32) {
    double d = std::ceil(delta);
    if (d < 1) d = 1;
    if (d >= 4294967296.0) return DELTA_INF;
    return (unsigned long long)d;
  }
  float f = (float)delta;
  if (!(f > 0.0f)) f = 1.17549435e-38f;  // smallest normal
  if (std::isinf(f)) return DELTA_INF;
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}

// Defaults when neither the caller nor the autotune cache sets them.  Dense
// low-diameter graphs (average degree >= 8) take narrow buckets (half the
// mean arc cost) and 4096-vertex blocks; sparse ones, typically of high
// diameter with thin frontiers, take wide buckets (16 mean costs) so that a
// bucket spans many hops, and 65536-vertex blocks.
static bool dense_graph(int n, long long m) { return n > 0 && m >= 8ll * n; }

float auto_delta_factor(int n, long long m) { return dense_graph(n, m) ? 0.5f : 16.0f; }

int default_parts(int n, long long m) {
  const long long b = dense_graph(n, m) ? 4096 : 65536;
  long long p = ((long long)n + b - 1) / b;
  if (p < 1) p = 1;
  if (p > 65536) p = 65536;
  return (int)p;
}

SolvePlan make_plan(const sssp_csr &g, const sssp_opts &o) {
  SolvePlan pl;
  sssp_opts tuned;
  bool have = false;
  if (!(o.flags & SSSP_F_NO_AUTOTUNE) &&
      (o.delta == 0 || o.num_partitions == 0 || o.wg_size == 0 || o.lag == 0))
    have = autotune_lookup(g, &tuned);
  const double delta = o.delta != 0 ? o.delta : (have ? tuned.delta : 0.0);
  int P = o.num_partitions > 0 ? o.num_partitions
                               : (have && tuned.num_partitions > 0 ? tuned.num_partitions
                                                                   : default_parts(g.n, g.m));
  if (P > g.n) P = g.n;
  const int pmin = (int)(((long long)g.n + 65535) / 65536);  // blocks <= 65536 vertices
  if (P < pmin) P = pmin;
  pl.bsize = (g.n + P - 1) / P;
  pl.nparts = (g.n + pl.bsize - 1) / pl.bsize;  // non-empty blocks only
  if (delta != 0) {
    pl.delta = delta_units(delta, g.wtype);
  } else {
    pl.delta = DELTA_AUTO;
    pl.auto_factor = auto_delta_factor(g.n, g.m);
  }
  // dense graphs: one 512-thread workgroup per CU (more workers mostly add
  // contention on the unit tables and labels); sparse, high-diameter graphs
  // with thin frontiers: two 256-thread workgroups per CU
  const bool dense = dense_graph(g.n, g.m);
  pl.bs = o.wg_size ? o.wg_size : (have && tuned.wg_size ? tuned.wg_size : (dense ? 512 : 256));
  pl.grid_per_cu = dense ? 1 : 2;
  pl.grid = o.num_workgroups ? o.num_workgroups
                             : (have && tuned.num_workgroups ? tuned.num_workgroups : 0);
  pl.lag = o.lag ? o.lag : (have ? tuned.lag : 0);
  return pl;
}

// Persistent grid: the requested size (0 = per_cu workgroups per CU), capped
// by what can be resident at block size bs.
int plan_grid(int wtype, int bs, int want, int per_cu_default, int mode) {
  const DevInfo di = device_info();
  const int per_cu = solve_max_blocks_per_cu(wtype, bs, mode);
  const int resident = di.cus * per_cu;
  if (want <= 0) want = di.cus * per_cu_default;
  int grid = want < resident ? want : resident;
  return grid < 1 ? 1 : grid;
}

// Solve mode (k_solve's local rule and update path) chosen by the flags.
int solve_mode(uint32_t flags) {
  if (flags & SSSP_F_IDLE_PRUNE) return SOLVE_IDLE_PRUNE;
  if (flags & SSSP_F_LOCAL_HEAP) return SOLVE_HEAP;
  if (flags & SSSP_F_BUFFER_CROSS) return SOLVE_BUFFERED;
  return SOLVE_BUCKETS;
}

// Workspace layout of a (batched) solve.
struct SolveLayout {
  size_t desc = 0, unit_solve = 0, unit_min = 0, abits = 0, ctrl = 0, keep = 0, total = 0;
  std::vector<size_t> label, dirty;
};

// keep_arcs > 0: one keep bit per arc for idle-time pruning (single solve).
SolveLayout solve_layout(int nsolves, const std::vector<int> &ns, int nunits, int keep_arcs = 0) {
  SolveLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes ? bytes : 1, 256);
    return at;
  };
  const int nabw = (nunits + ABW_UNITS - 1) / ABW_UNITS;
  L.ctrl = take(sizeof(Ctrl));
  L.desc = take(sizeof(SolveDesc) * (size_t)nsolves);
  L.unit_solve = take(sizeof(int32_t) * (size_t)nunits);
  L.unit_min = take(sizeof(unsigned long long) * (size_t)nunits);
  L.abits = take(sizeof(uint32_t) * ABW_STRIDE * (size_t)nabw);
  L.label.resize(nsolves);
  L.dirty.resize(nsolves);
  for (int i = 0; i < nsolves; i++) {
    L.label[i] = take(sizeof(unsigned long long) * (size_t)ns[i]);
    L.dirty[i] = take(sizeof(uint32_t) * (size_t)((ns[i] + 31) / 32));
  }
  if (keep_arcs > 0) L.keep = take(sizeof(uint32_t) * (size_t)((keep_arcs + 31) / 32));
  L.total = off;
  return L;
}

// lag * delta in distance units: an integer, or the fp32 bits of lag * delta.
unsigned long long window_units(unsigned long long delta, unsigned long long lag, int wtype) {
  if (wtype == SSSP_W_U32) {
    const unsigned long long w = delta * lag;
    return w / lag == delta ? w : DELTA_INF;
  }
  float d;
  uint32_t b = (uint32_t)delta;
  std::memcpy(&d, &b, 4);
  const float w = d * (float)lag;
  uint32_t wb;
  std::memcpy(&wb, &w, 4);
  return wb;
}

thread_local double g_solve_time_limit_s = 30.0;

unsigned long long time_limit_ticks(double seconds) {
  return (unsigned long long)(seconds * (double)device_info().wall_khz * 1000.0);
}

// Enqueues the whole solve sequence for prepared descriptors.
int run_solves(std::vector<SolveDesc> &descs, const SolveLayout &L, int nunits, int wtype,
               int bs, int grid, const sssp_opts &o, const sssp_csr *validate_graphs,
               int nvalidate, sssp_stats *stats, char *ws, hipStream_t st) {
  SolveArgs a;
  std::memset(&a, 0, sizeof(a));
  a.desc = reinterpret_cast<const SolveDesc *>(ws + L.desc);
  a.unit_solve = reinterpret_cast<int32_t *>(ws + L.unit_solve);
  a.unit_min = reinterpret_cast<unsigned long long *>(ws + L.unit_min);
  a.abits = reinterpret_cast<uint32_t *>(ws + L.abits);
  a.ctrl = reinterpret_cast<Ctrl *>(ws + L.ctrl);
  a.stats = stats;
  a.nunits = nunits;
  a.nabw = (nunits + ABW_UNITS - 1) / ABW_UNITS;
  a.max_rounds = o.max_rounds;
  a.num_solves = (int)descs.size();
  a.window = DELTA_INF;
  a.auto_lag = 0;
  if (solve_mode(o.flags) == SOLVE_IDLE_PRUNE && descs.size() == 1 && descs[0].m > 0) {
    a.keepbits = reinterpret_cast<uint32_t *>(ws + L.keep);
    a.keep_out = static_cast<uint8_t *>(o.keep_out);
    a.desc_m0 = descs[0].m;
    a.prune_tasks = (descs[0].n + PRUNE_CHUNK - 1) / PRUNE_CHUNK;
  }
  if (descs.size() == 1 && o.lag >= 0 && descs[0].delta != DELTA_INF) {
    const unsigned long long lag = o.lag > 0 ? (unsigned long long)o.lag : 1ull;
    if (descs[0].delta == DELTA_AUTO) a.auto_lag = (int)lag;
    else a.window = window_units(descs[0].delta, lag, wtype);
  }
  bool any_auto = false;
  for (const SolveDesc &d : descs) any_auto = any_auto || d.delta == DELTA_AUTO;
  a.time_limit = time_limit_ticks(g_solve_time_limit_s);

  const int ns = (int)descs.size();
  int max_n = 1;
  for (int i = 0; i < ns; i++) max_n = descs[i].n > max_n ? descs[i].n : max_n;
  for (int first = 0; first < ns; first += 32) {
    DescChunk c;
    std::memset(&c, 0, sizeof(c));
    c.first = first;
    c.count = ns - first < 32 ? ns - first : 32;
    for (int i = 0; i < c.count; i++) c.d[i] = descs[first + i];
    if (launch_write_desc(c, reinterpret_cast<SolveDesc *>(ws + L.desc), st) != hipSuccess)
      return SSSP_ERR_HIP;
  }
  if (launch_init(a, ns, max_n, st) != hipSuccess) return SSSP_ERR_HIP;
  if (any_auto && launch_auto_delta(a, wtype, ns, st) != hipSuccess) return SSSP_ERR_HIP;
  if (o.flags & SSSP_F_VALIDATE)
    for (int i = 0; i < nvalidate; i++)
      if (launch_validate(validate_graphs[i], 0, 0, &a.ctrl->status, st) != hipSuccess)
        return SSSP_ERR_HIP;
  // k_init ran before the validation above; the solve kernel checks status.
  if (o.event_start && hipEventRecord((hipEvent_t)o.event_start, st) != hipSuccess)
    return SSSP_ERR_HIP;
  if (launch_solve(a, wtype, bs, solve_mode(o.flags), grid, st) != hipSuccess)
    return SSSP_ERR_HIP;
  if (o.event_stop && hipEventRecord((hipEvent_t)o.event_stop, st) != hipSuccess)
    return SSSP_ERR_HIP;
  if (launch_epilogue(a, wtype, ns, max_n, st) != hipSuccess) return SSSP_ERR_HIP;
  if (a.keep_out && launch_keep_out(a, st) != hipSuccess) return SSSP_ERR_HIP;
  if (o.flags & SSSP_F_SYNC) return finish_sync(&a.ctrl->status, st);
  return SSSP_OK;
}

}  // namespace sssp_impl

// =================================================================== C ABI
extern "C" const char *sssp_strerror(int code) { return strerror_impl(code); }

extern "C" void sssp_opts_init(sssp_opts *o) {
  if (o) std::memset(o, 0, sizeof(*o));
}

extern "C" const char *sssp_version(void) { return "sssp-mi355x 0.1.0 (gfx950)"; }

extern "C" int sssp_solve(const sssp_csr *g, int32_t source, const sssp_opts *o, void *dist,
                          int32_t *pred, int32_t *pred_edge, sssp_stats *stats, void *ws,
                          size_t *ws_bytes, void *stream) {
  int rc = check_csr(g);
  if (rc) return rc;
  if (!ws_bytes) return SSSP_ERR_ARG;
  sssp_opts opts;
  sssp_opts_init(&opts);
  if (o) opts = *o;
  if ((rc = check_opts(&opts))) return rc;
  if (source < 0 || source >= g->n) return SSSP_ERR_SOURCE;
  const SolvePlan pl = make_plan(*g, opts);
  const bool iprune = solve_mode(opts.flags) == SOLVE_IDLE_PRUNE;
  const SolveLayout L = solve_layout(1, std::vector<int>{g->n}, pl.nparts, iprune ? g->m : 0);
  if (!ws) {
    *ws_bytes = L.total;
    return SSSP_OK;
  }
  if (!dist) return SSSP_ERR_ARG;
  if ((rc = check_ws(ws, *ws_bytes, L.total))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_sync(opts, st))) return rc;
  char *w = static_cast<char *>(ws);
  std::vector<SolveDesc> descs(1);
  SolveDesc &d = descs[0];
  std::memset(&d, 0, sizeof(d));
  d.row_ptr = g->row_ptr;
  d.col = g->col;
  d.w = static_cast<const uint32_t *>(g->w);
  d.label = reinterpret_cast<unsigned long long *>(w + L.label[0]);
  d.dirty = reinterpret_cast<uint32_t *>(w + L.dirty[0]);
  d.dist = dist;
  d.pred = pred;
  d.pred_edge = pred_edge;
  d.delta = pl.delta;
  d.auto_factor = pl.auto_factor;
  d.n = g->n;
  d.m = g->m;
  d.source = source;
  d.nparts = pl.nparts;
  d.bsize = pl.bsize;
  d.unit0 = 0;
  d.nwords = (g->n + 31) / 32;
  opts.lag = pl.lag;
  return run_solves(descs, L, pl.nparts, g->wtype, pl.bs,
                    plan_grid(g->wtype, pl.bs, pl.grid, pl.grid_per_cu, solve_mode(opts.flags)),
                    opts, g, 1, stats, w, st);
}

extern "C" int sssp_solve_batch(int32_t num_graphs, const sssp_csr *graphs, int32_t num_solves,
                                const int32_t *solve_graph, const int32_t *solve_source,
                                const int64_t *out_offset, const sssp_opts *o, void *dist,
                                int32_t *pred, int32_t *pred_edge, sssp_stats *stats, void *ws,
                                size_t *ws_bytes, void *stream) {
  if (num_graphs < 1 || num_solves < 1 || num_solves > 65535 || !graphs || !solve_graph ||
      !solve_source || !out_offset || !ws_bytes)
    return SSSP_ERR_ARG;
  if (o && (o->flags & SSSP_F_IDLE_PRUNE)) return SSSP_ERR_ARG;  // single solves only
  int rc;
  for (int i = 0; i < num_graphs; i++) {
    if ((rc = check_csr(&graphs[i]))) return rc;
    if (graphs[i].wtype != graphs[0].wtype) return SSSP_ERR_ARG;
  }
  sssp_opts opts;
  sssp_opts_init(&opts);
  if (o) opts = *o;
  if ((rc = check_opts(&opts))) return rc;
  // automatic fields come from the batch's own cache entry (entries tuned
  // for single solves do not carry over: a batch runs without a lag window)
  if (!(opts.flags & SSSP_F_NO_AUTOTUNE)) {
    sssp_opts tuned;
    if (autotune_lookup_batch(num_graphs, graphs, num_solves, &tuned)) {
      if (opts.delta == 0) opts.delta = tuned.delta;
      if (opts.num_partitions == 0) opts.num_partitions = tuned.num_partitions;
      if (opts.wg_size == 0) opts.wg_size = tuned.wg_size;
      if (opts.num_workgroups == 0) opts.num_workgroups = tuned.num_workgroups;
    }
    opts.flags |= SSSP_F_NO_AUTOTUNE;
  }
  std::vector<SolvePlan> gplan(num_graphs);
  for (int i = 0; i < num_graphs; i++) gplan[i] = make_plan(graphs[i], opts);
  std::vector<int> ns(num_solves);
  long long nunits = 0;
  for (int s = 0; s < num_solves; s++) {
    const int gi = solve_graph[s];
    if (gi < 0 || gi >= num_graphs) return SSSP_ERR_ARG;
    if (solve_source[s] < 0 || solve_source[s] >= graphs[gi].n) return SSSP_ERR_SOURCE;
    if (out_offset[s] < 0) return SSSP_ERR_ARG;
    ns[s] = graphs[gi].n;
    nunits += gplan[gi].nparts;
  }
  if (nunits > (1 << 30)) return SSSP_ERR_ARG;
  const SolveLayout L = solve_layout(num_solves, ns, (int)nunits);
  if (!ws) {
    *ws_bytes = L.total;
    return SSSP_OK;
  }
  if (!dist) return SSSP_ERR_ARG;
  if ((rc = check_ws(ws, *ws_bytes, L.total))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_sync(opts, st))) return rc;
  char *w = static_cast<char *>(ws);
  const size_t esz = 4;
  std::vector<SolveDesc> descs(num_solves);
  int unit0 = 0, bs = 0, grid = 0;
  for (int s = 0; s < num_solves; s++) {
    const int gi = solve_graph[s];
    const sssp_csr &g = graphs[gi];
    const SolvePlan &pl = gplan[gi];
    SolveDesc &d = descs[s];
    std::memset(&d, 0, sizeof(d));
    d.row_ptr = g.row_ptr;
    d.col = g.col;
    d.w = static_cast<const uint32_t *>(g.w);
    d.label = reinterpret_cast<unsigned long long *>(w + L.label[s]);
    d.dirty = reinterpret_cast<uint32_t *>(w + L.dirty[s]);
    d.dist = static_cast<char *>(dist) + esz * (size_t)out_offset[s];
    d.pred = pred ? pred + out_offset[s] : nullptr;
    d.pred_edge = pred_edge ? pred_edge + out_offset[s] : nullptr;
    d.delta = pl.delta;
    d.auto_factor = pl.auto_factor;
    d.n = g.n;
    d.m = g.m;
    d.source = solve_source[s];
    d.nparts = pl.nparts;
    d.bsize = pl.bsize;
    d.unit0 = unit0;
    d.nwords = (g.n + 31) / 32;
    unit0 += pl.nparts;
    bs = bs > pl.bs ? bs : pl.bs;
    grid = grid > pl.grid ? grid : pl.grid;
  }
  if (opts.wg_size) bs = opts.wg_size;
  // the grid follows the largest per-graph plan, capped by residency at bs
  if (opts.num_workgroups) grid = opts.num_workgroups;
  grid = plan_grid(graphs[0].wtype, bs, grid, 1, solve_mode(opts.flags));
  return run_solves(descs, L, (int)nunits, graphs[0].wtype, bs, grid, opts, graphs, num_graphs,
                    stats, w, st);
}

extern "C" int sssp_prune(const sssp_csr *g, const sssp_opts *o, uint8_t *keep,
                          int32_t *out_row_ptr, int32_t *out_col, void *out_w, int32_t *edge_map,
                          sssp_stats *stats, void *ws, size_t *ws_bytes, void *stream) {
  int rc = check_csr(g);
  if (rc) return rc;
  if (!ws_bytes) return SSSP_ERR_ARG;
  sssp_opts opts;
  sssp_opts_init(&opts);
  if (o) opts = *o;
  if ((rc = check_opts(&opts))) return rc;
  const int nset = (out_row_ptr != nullptr) + (out_col != nullptr) + (out_w != nullptr) +
                   (edge_map != nullptr);
  if (nset != 0 && nset != 4) return SSSP_ERR_ARG;
  const bool compact = nset == 4;
  const size_t need = prune_ws_bytes(g->n, g->m, compact);
  if (!ws) {
    *ws_bytes = need;
    return SSSP_OK;
  }
  if (!keep && g->m > 0) return SSSP_ERR_ARG;
  if ((rc = check_ws(ws, *ws_bytes, need))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_sync(opts, st))) return rc;
  int P = opts.num_partitions > 0 ? opts.num_partitions : default_parts(g->n, g->m);
  if (P > g->n) P = g->n;
  const int bsize = (g->n + P - 1) / P;
  const int local = (opts.flags & SSSP_F_PRUNE_LOCAL) ? 1 : 0;
  int32_t *dev_status = nullptr;
  const bool hubs = !(opts.flags & SSSP_F_PRUNE_NO_HUBS);
  rc = launch_prune(*g, local, hubs, bsize, keep, out_row_ptr, out_col, out_w, edge_map, stats,
                    static_cast<char *>(ws), device_info().cus,
                    (opts.flags & SSSP_F_VALIDATE) != 0, opts.event_start, opts.event_stop,
                    &dev_status, st);
  if (rc) return rc;
  if (opts.flags & SSSP_F_SYNC) return finish_sync(dev_status, st);
  return SSSP_OK;
}

extern "C" int sssp_backward(const sssp_csr *g, int32_t source, const float *dist,
                             const int32_t *pred_edge, const float *grad_dist, float *grad_w,
                             const sssp_opts *o, sssp_stats *stats, void *ws, size_t *ws_bytes,
                             void *stream) {
  int rc = check_csr(g);
  if (rc) return rc;
  if (g->wtype != SSSP_W_F32 || !ws_bytes) return SSSP_ERR_ARG;
  sssp_opts opts;
  sssp_opts_init(&opts);
  if (o) opts = *o;
  if ((rc = check_opts(&opts))) return rc;
  if (source < 0 || source >= g->n) return SSSP_ERR_SOURCE;
  const size_t need = backward_ws_bytes(g->n);
  if (!ws) {
    *ws_bytes = need;
    return SSSP_OK;
  }
  if (!dist || !pred_edge || !grad_dist || (!grad_w && g->m > 0)) return SSSP_ERR_ARG;
  if ((rc = check_ws(ws, *ws_bytes, need))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_sync(opts, st))) return rc;
  int32_t *dev_status = nullptr;
  if (opts.event_start && hipEventRecord((hipEvent_t)opts.event_start, st) != hipSuccess)
    return SSSP_ERR_HIP;
  rc = launch_backward(*g, source, dist, pred_edge, grad_dist, grad_w,
                       (opts.flags & SSSP_F_VALIDATE) != 0, stats, static_cast<char *>(ws),
                       &dev_status, st);
  if (rc) return rc;
  if (opts.event_stop && hipEventRecord((hipEvent_t)opts.event_stop, st) != hipSuccess)
    return SSSP_ERR_HIP;
  if (opts.flags & SSSP_F_SYNC) return finish_sync(dev_status, st);
  return SSSP_OK;
}
