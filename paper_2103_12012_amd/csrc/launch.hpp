// launch.hpp -- host-side launchers of the library's kernels.
#pragma once
#include "internal.hpp"

namespace sssp_impl {

// solve.hip
hipError_t launch_validate(const sssp_csr &g, int need_sorted, int need_positive,
                           int32_t *status, hipStream_t st);
hipError_t launch_write_desc(const DescChunk &c, SolveDesc *table, hipStream_t st);
hipError_t launch_init(const SolveArgs &a, int nsolves, int max_n, hipStream_t st);
hipError_t launch_auto_delta(const SolveArgs &a, int wtype, int nsolves, hipStream_t st);
hipError_t launch_solve(const SolveArgs &a, int wtype, int bs, int mode, int grid,
                        hipStream_t st);
hipError_t launch_keep_out(const SolveArgs &a, hipStream_t st);
hipError_t launch_epilogue(const SolveArgs &a, int wtype, int nsolves, int max_n,
                           hipStream_t st);
int solve_max_blocks_per_cu(int wtype, int bs, int mode);
__global__ void k_copy_status(const int32_t *status, sssp_stats *stats);

// scan.hip
size_t scan_tmp_bytes(int n);
hipError_t launch_excl_scan(const int32_t *in, int n, int32_t *out, int32_t *tmp,
                            hipStream_t st);
// In-place exclusive scan of ntiles tile totals by one workgroup (the
// second step of a tiled scan); *total = their sum.  Tiles of a scan hold
// SCAN_TILE elements.
constexpr int SCAN_TILE = 2048;
hipError_t launch_scan_sums(int32_t *tile_sum, int ntiles, int32_t *total, hipStream_t st);

// prune.hip
size_t prune_ws_bytes(int n, int m, bool compact);
int launch_prune(const sssp_csr &g, int local, bool hubs, int bsize, uint8_t *keep,
                 int32_t *out_row_ptr,
                 int32_t *out_col, void *out_w, int32_t *edge_map, sssp_stats *stats,
                 char *ws, int grid_cus, bool validate, void *ev_start, void *ev_stop,
                 int32_t **status_out, hipStream_t st);

// backward.hip
size_t backward_ws_bytes(int n);
int launch_backward(const sssp_csr &g, int source, const float *dist, const int32_t *pred_edge,
                    const float *grad_dist, float *grad_w, bool validate, sssp_stats *stats,
                    char *ws, int32_t **status_out, hipStream_t st);

}  // namespace sssp_impl
