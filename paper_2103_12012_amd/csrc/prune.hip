// prune.hip -- Trishla triangle pruning (Sec. III-B, Alg. 1) on gfx950.
//
// Arc e = (u,x,W) is deleted when some middle y, y != u and y != x, has arcs
// (u,y,w1), (y,x,w2) with w1 + w2 < W, tested against the input graph for
// all arcs at once.  For a row u the kernel keeps, per target x of u, the
// cheapest two-arc cost best[x] = min_y w(u,y) + w(y,x) in an LDS hash
// table, streams every middle's sorted row N(y) restricted to the target
// range of the table (binary search on the sorted row), and finally compares
// every arc of u against best[x].
//
// Work per row is sum over its middles of |N(y)|, which is highly skewed on
// power-law graphs, so rows are split into items: nx chunks of at most XCAP
// consecutive targets (a key range, since rows are sorted) times ny
// interleaved subsets of the middles.  Items of a row split over middles
// combine their minima with a 64-bit atomic min per arc in HBM; the last of
// them to finish (a per-chunk counter) writes the keep flags.
//
// Integer costs are summed in 64 bits; fp32 costs are summed in double,
// which decides w1 + w2 < W exactly for fp32 operands (the sum is exact
// unless one operand is below 2^-29 of the other, and then the comparison
// with an fp32 W cannot flip).
#include "internal.hpp"
#include "launch.hpp"

namespace sssp_impl {

constexpr int TRI_BS = 512;
constexpr int TRI_XCAP = 2048;              // targets per table chunk
constexpr int TRI_HCAP = 4096;              // hash slots, >= 2 * XCAP
constexpr int TRI_YCAP = 1024;              // middles staged per round
constexpr long long TRI_TARGET = 1ll << 20; // wedges per item
constexpr int TRI_NYMAX = 1024;
constexpr int TRI_LIGHT_CHUNK = 16;         // light rows taken per ticket
constexpr unsigned long long KEY_INF = ~0ull;

template <int WT> struct TriCost;
template <> struct TriCost<SSSP_W_U32> {
  __device__ static __forceinline__ unsigned long long key(uint32_t w) { return w; }
  __device__ static __forceinline__ unsigned long long sum(unsigned long long k1, uint32_t w2) {
    return k1 + w2;
  }
};
template <> struct TriCost<SSSP_W_F32> {
  __device__ static __forceinline__ unsigned long long key(uint32_t w) {
    return (unsigned long long)__double_as_longlong((double)__uint_as_float(w));
  }
  __device__ static __forceinline__ unsigned long long sum(unsigned long long k1, uint32_t w2) {
    const double s = __longlong_as_double((long long)k1) + (double)__uint_as_float(w2);
    return (unsigned long long)__double_as_longlong(s);
  }
};

struct TriArgs {
  const int32_t *row_ptr;
  const int32_t *col;
  const uint32_t *w;
  int n, m, local, bsize;
  uint8_t *keep;
  unsigned long long *gbest;  // per arc: cheapest detour, for split rows
  int32_t *chunk_done;        // per arc (first arc of a chunk): finished items
  int32_t *ny;                // per row: middle subsets (0 = empty row)
  int32_t *nitems;            // per row: nx * ny
  int32_t *flag;              // per row: 1 when split (nitems > 1)
  int32_t *hpos;              // exclusive scan of flag (n+1): heavy row index
  int32_t *heavy_u;           // heavy rows in order
  int32_t *hitems;            // items of heavy row i
  int32_t *hoff;              // exclusive scan of hitems
  int32_t *tickets;           // [0] light, [1] heavy
  int32_t *status;
  sssp_stats *stats;
};

// ------------------------------------------------------------------ plan
// One wave per row: W(u) = sum over middles y of |N(y)|, then the split.
__global__ void k_tri_plan(TriArgs a) {
  if (*a.status) return;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nwaves = gridDim.x * blockDim.x / WAVE;
  const int lane = lane_id();
  for (int u = wave; u < a.n; u += nwaves) {
    const int rs = a.row_ptr[u], re = a.row_ptr[u + 1];
    const int deg = re - rs;
    long long wsum = 0;
    for (int e = rs + lane; e < re; e += WAVE) {
      const int y = a.col[e];
      if (y == u || (unsigned)y >= (unsigned)a.n) continue;
      if (a.local && y / a.bsize != u / a.bsize) continue;
      wsum += a.row_ptr[y + 1] - a.row_ptr[y];
    }
    wsum = wave_sum(wsum);
    if (lane == 0) {
      int nyv = 0, items = 0;
      if (deg > 0) {
        const int nx = (deg + TRI_XCAP - 1) / TRI_XCAP;
        long long want = (wsum + (long long)nx * TRI_TARGET - 1) / ((long long)nx * TRI_TARGET);
        long long cap = deg < TRI_NYMAX ? deg : TRI_NYMAX;
        if (want > cap) want = cap;
        nyv = want < 1 ? 1 : (int)want;
        items = nx * nyv;
      }
      a.ny[u] = nyv;
      a.nitems[u] = items;
      a.flag[u] = items > 1;
    }
  }
}

__global__ void k_tri_heavy_list(TriArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int u = t; u < a.n; u += stride)
    if (a.flag[u]) {
      const int i = a.hpos[u];
      a.heavy_u[i] = u;
      a.hitems[i] = a.nitems[u];
    }
}

__global__ void k_tri_init(TriArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < a.m; e += stride) {
    a.gbest[e] = KEY_INF;
    a.chunk_done[e] = 0;
  }
  for (int i = t; i < a.n; i += stride) a.hitems[i] = 0;
  if (t == 0) {
    a.tickets[0] = 0;
    a.tickets[1] = 0;
    *a.status = 0;
  }
  if (a.stats && t < (int)(sizeof(sssp_stats) / 4))
    reinterpret_cast<uint32_t *>(a.stats)[t] = 0u;
}

// ------------------------------------------------------------------ items
struct TriShared {
  int32_t key[TRI_HCAP];
  unsigned long long best[TRI_HCAP];
  int32_t y_beg[TRI_YCAP];
  int32_t y_off[TRI_YCAP + 1];
  int32_t y_id[TRI_YCAP];
  unsigned long long y_w1[TRI_YCAP];
  int ws[TRI_BS / WAVE + 1];
  int flag;
};

__device__ __forceinline__ uint32_t tri_hash(int x, int hbits) {
  return ((uint32_t)x * 2654435761u) >> (32 - hbits);
}

__device__ __forceinline__ int tri_lower(const int32_t *col, int lo, int hi, int x) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int tri_upper(const int32_t *col, int lo, int hi, int x) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <int WT>
__device__ void tri_item(const TriArgs &a, TriShared &sh, int u, int xc, int yp, int ny) {
  constexpr int BS = TRI_BS;
  constexpr int EPT = TRI_YCAP / BS;
  const int tid = threadIdx.x;
  const int rs = a.row_ptr[u];
  const int deg = a.row_ptr[u + 1] - rs;
  const int cs = xc * TRI_XCAP;
  const int ce = min(deg, cs + TRI_XCAP);
  const int clen = ce - cs;
  int hbits = 6;
  while ((1 << hbits) < 2 * clen) hbits++;
  const int hs = 1 << hbits;
  const int hmask = hs - 1;

  for (int i = tid; i < hs; i += BS) {
    sh.key[i] = -1;
    sh.best[i] = KEY_INF;
  }
  __syncthreads();
  for (int j = tid; j < clen; j += BS) {
    const int x = a.col[rs + cs + j];
    uint32_t h = tri_hash(x, hbits);
    for (;;) {
      const int old = atomicCAS(&sh.key[h], -1, x);
      if (old == -1 || old == x) break;
      h = (h + 1) & hmask;
    }
  }
  __syncthreads();

  const int xlo = a.col[rs + cs];
  const int xhi = a.col[rs + ce - 1];
  const int nmid = deg > yp ? (deg - yp + ny - 1) / ny : 0;
  const int part_u = u / a.bsize;
  long long wedges = 0;
  for (int mb = 0; mb < nmid; mb += TRI_YCAP) {
    const int cnt = min(TRI_YCAP, nmid - mb);
    int lens[EPT];
    int lsum = 0;
#pragma unroll
    for (int jj = 0; jj < EPT; jj++) {
      const int k = tid * EPT + jj;
      int len = 0;
      if (k < cnt) {
        const int e1 = rs + yp + (mb + k) * ny;
        const int y = a.col[e1];
        if (y != u && (unsigned)y < (unsigned)a.n && (!a.local || y / a.bsize == part_u)) {
          const int ya = a.row_ptr[y], yb = a.row_ptr[y + 1];
          const int lo = tri_lower(a.col, ya, yb, xlo);
          const int hi = tri_upper(a.col, lo, yb, xhi);
          sh.y_beg[k] = lo;
          sh.y_id[k] = y;
          sh.y_w1[k] = TriCost<WT>::key(a.w[e1]);
          len = hi - lo;
        } else {
          sh.y_beg[k] = 0;
          sh.y_id[k] = -1;
          sh.y_w1[k] = 0;
        }
      }
      lens[jj] = len;
      lsum += len;
    }
    int tot;
    int run = block_excl_scan<BS>(lsum, sh.ws, &tot);
#pragma unroll
    for (int jj = 0; jj < EPT; jj++) {
      const int k = tid * EPT + jj;
      if (k < cnt) sh.y_off[k] = run;
      run += lens[jj];
    }
    if (tid == 0) sh.y_off[cnt] = tot;
    __syncthreads();
    for (int idx = tid; idx < tot; idx += BS) {
      int lo = 0, hi = cnt - 1;  // last k with y_off[k] <= idx
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sh.y_off[mid] <= idx) lo = mid;
        else hi = mid - 1;
      }
      const int f = sh.y_beg[lo] + (idx - sh.y_off[lo]);
      const int x = a.col[f];
      if (x == sh.y_id[lo]) continue;
      uint32_t h = tri_hash(x, hbits);
      for (;;) {
        const int k2 = sh.key[h];
        if (k2 == x) {
          atomicMin(&sh.best[h], TriCost<WT>::sum(sh.y_w1[lo], a.w[f]));
          break;
        }
        if (k2 == -1) break;
        h = (h + 1) & hmask;
      }
    }
    wedges += tot;
    __syncthreads();
  }

  // flush: compare every arc of the chunk with its cheapest detour
  unsigned int pruned = 0;
  for (int j = tid; j < clen; j += BS) {
    const int e = rs + cs + j;
    const int x = a.col[e];
    uint32_t h = tri_hash(x, hbits);
    while (sh.key[h] != x) h = (h + 1) & hmask;
    const unsigned long long b = sh.best[h];
    if (ny == 1) {
      const bool del = b < TriCost<WT>::key(a.w[e]);
      a.keep[e] = del ? 0 : 1;
      pruned += del;
    } else if (b != KEY_INF) {
      amin(&a.gbest[e], b);
    }
  }
  if (ny > 1) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      const int prev = aadd(&a.chunk_done[rs + cs], 1);
      sh.flag = prev == ny - 1;
    }
    __syncthreads();
    if (sh.flag) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      for (int j = tid; j < clen; j += BS) {
        const int e = rs + cs + j;
        const bool del = ld_rlx(&a.gbest[e]) < TriCost<WT>::key(a.w[e]);
        a.keep[e] = del ? 0 : 1;
        pruned += del;
      }
    }
  }
  if (a.stats) {
    pruned = wave_sum(pruned);
    if (lane_id() == 0 && pruned) stat_add(&a.stats->edges_pruned, pruned);
    if (tid == 0 && wedges) stat_add(&a.stats->wedges, (uint64_t)wedges);
  }
  __syncthreads();
}

// Split rows first (item t -> heavy row i by binary search in hoff -> chunk
// and middle subset), then rows that fit one item, TRI_LIGHT_CHUNK
// consecutive rows per ticket.
template <int WT>
__global__ __launch_bounds__(TRI_BS) void k_tri_main(TriArgs a) {
  __shared__ TriShared sh;
  __shared__ int s_t;
  if (*a.status) return;
  const int nh = a.hpos[a.n];
  const int total = a.hoff[nh];
  for (;;) {
    if (threadIdx.x == 0) s_t = atomicAdd(&a.tickets[1], 1);
    __syncthreads();
    const int t = s_t;
    __syncthreads();
    if (t >= total) break;
    int lo = 0, hi = nh - 1;  // last i with hoff[i] <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.hoff[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int u = a.heavy_u[lo];
    const int ny = a.ny[u];
    const int local = t - a.hoff[lo];
    tri_item<WT>(a, sh, u, local / ny, local % ny, ny);
  }
  for (;;) {
    if (threadIdx.x == 0) s_t = atomicAdd(&a.tickets[0], TRI_LIGHT_CHUNK);
    __syncthreads();
    const int u0 = s_t;
    __syncthreads();
    if (u0 >= a.n) break;
    const int u1 = min(a.n, u0 + TRI_LIGHT_CHUNK);
    for (int u = u0; u < u1; u++)
      if (a.nitems[u] == 1) tri_item<WT>(a, sh, u, 0, 0, 1);
  }
}

// ------------------------------------------------------------ compaction
// One wave per row: kept-arc counts, then a stable ballot compaction.
__global__ void k_count_kept(const int32_t *row_ptr, const uint8_t *keep, int n, int32_t *cnt,
                             const int32_t *status) {
  if (*status) return;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nwaves = gridDim.x * blockDim.x / WAVE;
  for (int u = wave; u < n; u += nwaves) {
    int c = 0;
    for (int e = row_ptr[u] + lane_id(); e < row_ptr[u + 1]; e += WAVE) c += keep[e];
    c = wave_sum(c);
    if (lane_id() == 0) cnt[u] = c;
  }
}

__global__ void k_compact(const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                          const uint8_t *keep, int n, const int32_t *out_row_ptr,
                          int32_t *out_col, uint32_t *out_w, int32_t *edge_map,
                          const int32_t *status) {
  if (*status) return;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nwaves = gridDim.x * blockDim.x / WAVE;
  const int lane = lane_id();
  for (int u = wave; u < n; u += nwaves) {
    int pos = out_row_ptr[u];
    const int re = row_ptr[u + 1];
    for (int e0 = row_ptr[u]; e0 < re; e0 += WAVE) {
      const int e = e0 + lane;
      const bool k = e < re && keep[e];
      const unsigned long long bal = __ballot(k);
      const int before = __popcll(bal & ((1ull << lane) - 1ull));
      if (k) {
        out_col[pos + before] = col[e];
        out_w[pos + before] = w[e];
        edge_map[pos + before] = e;
      }
      pos += __popcll(bal);
    }
  }
}

// ------------------------------------------------------------ host side
size_t prune_ws_bytes(int n, int m, bool compact) {
  size_t b = 0;
  auto take = [&](size_t x) { b += align_up(x ? x : 1, 256); };
  take(8ull * m);              // gbest
  take(4ull * m);              // chunk_done
  for (int i = 0; i < 5; i++) take(4ull * (n + 1));  // ny, nitems, flag, hpos, heavy_u
  take(4ull * (n + 1));        // hitems
  take(4ull * (n + 2));        // hoff
  take(scan_tmp_bytes(n + 1)); // scan scratch
  take(256);                   // tickets + status
  if (compact) take(4ull * (n + 1));  // kept counts
  return b;
}

int launch_prune(const sssp_csr &g, int local, int bsize, uint8_t *keep, int32_t *out_row_ptr,
                 int32_t *out_col, void *out_w, int32_t *edge_map, sssp_stats *stats,
                 char *ws, int grid_cus, bool validate, int32_t **status_out,
                 hipStream_t st) {
  const int n = g.n, m = g.m;
  size_t off = 0;
  auto take = [&](size_t x) {
    char *p = ws + off;
    off += align_up(x ? x : 1, 256);
    return p;
  };
  TriArgs a;
  a.row_ptr = g.row_ptr;
  a.col = g.col;
  a.w = static_cast<const uint32_t *>(g.w);
  a.n = n;
  a.m = m;
  a.local = local;
  a.bsize = bsize;
  a.keep = keep;
  a.gbest = reinterpret_cast<unsigned long long *>(take(8ull * m));
  a.chunk_done = reinterpret_cast<int32_t *>(take(4ull * m));
  a.ny = reinterpret_cast<int32_t *>(take(4ull * (n + 1)));
  a.nitems = reinterpret_cast<int32_t *>(take(4ull * (n + 1)));
  a.flag = reinterpret_cast<int32_t *>(take(4ull * (n + 1)));
  a.hpos = reinterpret_cast<int32_t *>(take(4ull * (n + 1)));
  a.heavy_u = reinterpret_cast<int32_t *>(take(4ull * (n + 1)));
  a.hitems = reinterpret_cast<int32_t *>(take(4ull * (n + 1)));
  a.hoff = reinterpret_cast<int32_t *>(take(4ull * (n + 2)));
  int32_t *tmp = reinterpret_cast<int32_t *>(take(scan_tmp_bytes(n + 1)));
  char *misc = take(256);
  a.tickets = reinterpret_cast<int32_t *>(misc);
  a.status = reinterpret_cast<int32_t *>(misc + 16);
  a.stats = stats;
  int32_t *kept_cnt = out_row_ptr ? reinterpret_cast<int32_t *>(take(4ull * (n + 1))) : nullptr;
  *status_out = a.status;

  hipLaunchKernelGGL(k_tri_init, dim3(1024), dim3(256), 0, st, a);
  if (validate && launch_validate(g, 1, 0, a.status, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tri_plan, dim3(2048), dim3(256), 0, st, a);
  if (launch_excl_scan(a.flag, n, a.hpos, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tri_heavy_list, dim3(1024), dim3(256), 0, st, a);
  // hitems is zero beyond the heavy rows, so hoff[hpos[n]] is the total
  if (launch_excl_scan(a.hitems, n, a.hoff, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
  int per_cu = 0;
  if (g.wtype == SSSP_W_U32) {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tri_main<SSSP_W_U32>, TRI_BS, 0);
    hipLaunchKernelGGL(k_tri_main<SSSP_W_U32>, dim3(grid_cus * (per_cu > 0 ? per_cu : 1)),
                       dim3(TRI_BS), 0, st, a);
  } else {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tri_main<SSSP_W_F32>, TRI_BS, 0);
    hipLaunchKernelGGL(k_tri_main<SSSP_W_F32>, dim3(grid_cus * (per_cu > 0 ? per_cu : 1)),
                       dim3(TRI_BS), 0, st, a);
  }
  if (hipGetLastError() != hipSuccess) return SSSP_ERR_HIP;
  if (out_row_ptr) {
    hipLaunchKernelGGL(k_count_kept, dim3(2048), dim3(256), 0, st, g.row_ptr, keep, n, kept_cnt,
                       a.status);
    if (launch_excl_scan(kept_cnt, n, out_row_ptr, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
    hipLaunchKernelGGL(k_compact, dim3(2048), dim3(256), 0, st, g.row_ptr, g.col,
                       static_cast<const uint32_t *>(g.w), keep, n, out_row_ptr, out_col,
                       static_cast<uint32_t *>(out_w), edge_map, a.status);
  }
  hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st, a.status, stats);
  return hipGetLastError() == hipSuccess ? SSSP_OK : SSSP_ERR_HIP;
}

}  // namespace sssp_impl
