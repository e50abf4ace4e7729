// plan.hpp -- host-side helpers shared by the entry points.
#pragma once
#include "internal.hpp"

namespace sssp_impl {

struct DevInfo {
  int cus = 0;
  int wall_khz = 0;
};

// Parameters of one solve after defaults and the autotune cache are applied.
struct SolvePlan {
  int nparts = 1, bsize = 1;  // P (non-empty blocks) and block size ceil(n/P)
  int bs = 256, grid = 1;     // workgroup size and persistent grid (0 = default)
  int grid_per_cu = 1;        // default grid: workgroups per CU
  unsigned long long delta = DELTA_INF;  // DELTA_AUTO: set on the device
  float auto_factor = 0.0f;              // for DELTA_AUTO
  int lag = 0;                           // window in buckets (0 = default)
};

DevInfo device_info();
const char *strerror_impl(int code);
int check_csr(const sssp_csr *g);
int check_opts(const sssp_opts *o);
int check_ws(void *ws, size_t have, size_t need);
int check_sync(const sssp_opts &o, hipStream_t st);
int finish_sync(const int32_t *dev_status, hipStream_t st);
SolvePlan make_plan(const sssp_csr &g, const sssp_opts &o);
unsigned long long delta_units(double delta, int wtype);
int default_parts(int n, long long m);
float auto_delta_factor(int n, long long m);

// Device time limit of one solve launch in seconds (per host thread);
// sssp_autotune lowers it so that a slow candidate ends early.
extern thread_local double g_solve_time_limit_s;

// autotune.hip: cached best options for graphs of this signature, if any,
// and for a batch of this signature.
bool autotune_lookup(const sssp_csr &g, sssp_opts *out);
bool autotune_lookup_batch(int num_graphs, const sssp_csr *graphs, int num_solves,
                           sssp_opts *out);

}  // namespace sssp_impl
