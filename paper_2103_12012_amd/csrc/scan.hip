// scan.hip -- device-wide exclusive prefix sum of int32 (three kernels:
// tile scans, scan of tile totals, add tile offsets).  out has N+1 entries;
// out[N] is the total.
#include "internal.hpp"
#include "launch.hpp"

namespace sssp_impl {

constexpr int SCAN_BS = 256;
constexpr int SCAN_EPT = 8;
static_assert(SCAN_TILE == SCAN_BS * SCAN_EPT, "tile of the scans");

template <typename T>
__global__ __launch_bounds__(SCAN_BS) void k_scan_tiles(const T *in, int n, int32_t *out,
                                                        int32_t *tile_sum) {
  __shared__ int ws[SCAN_BS / WAVE + 1];
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_EPT;
  int v[SCAN_EPT];
  int s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_EPT; j++) {
    v[j] = base + j < n ? (int)in[base + j] : 0;
    s += v[j];
  }
  int tot;
  int run = block_excl_scan<SCAN_BS>(s, ws, &tot);
#pragma unroll
  for (int j = 0; j < SCAN_EPT; j++) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// One block scans the tile totals in chunks, carrying the running sum.
__global__ __launch_bounds__(SCAN_BS) void k_scan_sums(int32_t *tile_sum, int ntiles,
                                                       int32_t *out_total) {
  __shared__ int ws[SCAN_BS / WAVE + 1];
  int carry = 0;
  for (int c0 = 0; c0 < ntiles; c0 += SCAN_TILE) {
    const int base = c0 + threadIdx.x * SCAN_EPT;
    int v[SCAN_EPT];
    int s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_EPT; j++) {
      v[j] = base + j < ntiles ? tile_sum[base + j] : 0;
      s += v[j];
    }
    int tot;
    int run = block_excl_scan<SCAN_BS>(s, ws, &tot) + carry;
#pragma unroll
    for (int j = 0; j < SCAN_EPT; j++) {
      if (base + j < ntiles) tile_sum[base + j] = run;
      run += v[j];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *out_total = carry;
}

__global__ __launch_bounds__(SCAN_BS) void k_scan_add(int32_t *out, int n,
                                                      const int32_t *tile_off) {
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_EPT;
  const int add = tile_off[blockIdx.x];
#pragma unroll
  for (int j = 0; j < SCAN_EPT; j++)
    if (base + j < n) out[base + j] += add;
}

size_t scan_tmp_bytes(int n) {
  const int ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  return sizeof(int32_t) * (size_t)(ntiles > 0 ? ntiles : 1);
}

template <typename T>
static hipError_t excl_scan_t(const T *in, int n, int32_t *out, int32_t *tmp, hipStream_t st) {
  const int ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (ntiles > 0)
    hipLaunchKernelGGL(k_scan_tiles<T>, dim3(ntiles), dim3(SCAN_BS), 0, st, in, n, out, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BS), 0, st, tmp, ntiles, out + n);
  if (ntiles > 0)
    hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(SCAN_BS), 0, st, out, n, tmp);
  return hipGetLastError();
}

hipError_t launch_excl_scan(const int32_t *in, int n, int32_t *out, int32_t *tmp,
                            hipStream_t st) {
  return excl_scan_t(in, n, out, tmp, st);
}

hipError_t launch_scan_sums(int32_t *tile_sum, int ntiles, int32_t *total, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BS), 0, st, tile_sum, ntiles, total);
  return hipGetLastError();
}

}  // namespace sssp_impl
