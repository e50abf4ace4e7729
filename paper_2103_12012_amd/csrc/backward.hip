// backward.hip -- gradient of L = sum_v g[v] d(v) with respect to the arc
// costs, along the shortest-path tree given by pred_edge (fp32 graphs).
//
// d(t) is the sum of the costs on the tree path s -> t, so dL/dw_e is the
// total of g over the subtree hanging below e = pred_edge[v].  Subtree
// totals are formed in reverse distance order: a vertex is finalised only
// after all of its children (which lie strictly farther from s when every
// cost is positive).  Each vertex counts its unfinished children; a leaf
// starts a chain, adds its total into its parent (fp64 atomic add), and the
// child that brings the parent's count to zero continues the chain with the
// parent.  Every vertex is finalised exactly once, with no barrier between
// tree levels; a vertex never reached this way lies on a predecessor cycle.
//
// Only the part of the tree that carries gradient is walked: the vertices
// with g != 0 and their ancestors (marked by walking up from each such
// vertex, stopping at the first vertex already marked).  Every other arc's
// gradient is zero.  A sparse upstream gradient (a loss over a few targets)
// thus touches only the union of the targets' tree paths.
#include "internal.hpp"
#include "launch.hpp"

namespace sssp_impl {

struct BwdArgs {
  const int32_t *row_ptr;
  const int32_t *col;
  const float *dist;
  const int32_t *pred_edge;
  const float *g;
  float *grad_w;
  int n, m, source;
  int32_t *par;       // tail of pred_edge[v], -1 for the source / unreached
  int32_t *nchild;    // children not yet finalised
  int32_t *leaf;      // 1 when v starts a chain
  int32_t *mark;      // 1 when v carries gradient (g != 0 below it)
  double *acc;        // subtree totals
  unsigned long long *counts;  // [0] reached vertices != s, [1] finalised
  int32_t *status;
};

// Clears the gradient (and the per-vertex counters) even after a validation
// error, so the output never holds stale memory.
__global__ void k_bwd_zero(BwdArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < a.m; e += stride) a.grad_w[e] = 0.0f;
  for (int v = t; v < a.n; v += stride) {
    a.nchild[v] = 0;
    a.mark[v] = 0;
  }
  if (t == 0) {
    a.counts[0] = 0;
    a.counts[1] = 0;
  }
}

// Parent of every reached v != s (binary search of its pred arc's tail) and
// the starting totals acc[v] = g[v].
__global__ void k_bwd_parent(BwdArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int v = t; v < a.n; v += stride) {
    int p = -1;
    double g0 = 0.0;
    const float dv = a.dist[v];
    if (v != a.source && dv < __builtin_inff()) {
      const int pe = a.pred_edge[v];
      if (pe < 0 || pe >= a.m || a.col[pe] != v) {
        set_status(a.status, SSSP_ERR_ARG);
      } else {
        int lo = 0, hi = a.n - 1;  // largest u with row_ptr[u] <= pe
        while (lo < hi) {
          const int mid = lo + ((hi - lo + 1) >> 1);
          if (a.row_ptr[mid] <= pe) lo = mid;
          else hi = mid - 1;
        }
        p = lo;
        g0 = (double)a.g[v];
      }
    }
    a.par[v] = p;
    a.acc[v] = g0;
  }
}

// Marks every vertex with g != 0 and its ancestors: a walk up the tree stops
// at the source or at the first vertex some walk has marked already.  The
// number of marked vertices is counts[0].
__global__ void k_bwd_mark(BwdArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  unsigned long long marked = 0;
  for (int v = t; v < a.n; v += stride) {
    if (a.par[v] < 0 || a.acc[v] == 0.0) continue;
    int x = v;
    for (;;) {
      if (__hip_atomic_fetch_or(&a.mark[x], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      marked++;
      const int p = a.par[x];
      if (p == a.source || p < 0) break;
      x = p;
    }
  }
  marked = wave_sum(marked);
  if (lane_id() == 0 && marked) aadd(&a.counts[0], marked);
}

// Children that carry gradient, per parent.
__global__ void k_bwd_count(BwdArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int v = t; v < a.n; v += stride) {
    const int p = a.par[v];
    if (a.mark[v] && p >= 0 && p != a.source) atomicAdd(&a.nchild[p], 1);
  }
}

__global__ void k_bwd_leaves(BwdArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int v = t; v < a.n; v += stride) a.leaf[v] = a.mark[v] && a.par[v] >= 0 && a.nchild[v] == 0;
}

__global__ void k_bwd_chain(BwdArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  unsigned long long fin = 0;
  for (int v = t; v < a.n; v += stride) {
    if (!a.leaf[v]) continue;
    int x = v;
    for (;;) {
      const double tot = __hip_atomic_load(&a.acc[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a.grad_w[a.pred_edge[x]] = (float)tot;
      fin++;
      const int p = a.par[x];
      if (p == a.source || p < 0 || a.par[p] < 0) break;
      __hip_atomic_fetch_add(&a.acc[p], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int left = __hip_atomic_fetch_sub(&a.nchild[p], 1, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
      if (left != 1) break;  // a sibling is still pending; it continues later
      x = p;
    }
  }
  fin = wave_sum(fin);
  if (lane_id() == 0 && fin) aadd(&a.counts[1], fin);
}

__global__ void k_bwd_check(BwdArgs a, sssp_stats *stats) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (*a.status == 0 && a.counts[0] != a.counts[1]) set_status(a.status, SSSP_ERR_CYCLE);
    if (stats) stats->status = *a.status;
  }
}

__global__ void k_bwd_init_status(int32_t *status, sssp_stats *stats) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *status = 0;
    if (stats) {
      uint32_t *s = reinterpret_cast<uint32_t *>(stats);
      for (int i = 0; i < (int)(sizeof(sssp_stats) / 4); i++) s[i] = 0u;
    }
  }
}

size_t backward_ws_bytes(int n) {
  size_t b = 0;
  auto take = [&](size_t x) { b += align_up(x ? x : 1, 256); };
  take(4ull * n);
  take(4ull * n);
  take(4ull * n);
  take(4ull * n);
  take(8ull * n);
  take(256);
  return b;
}

int launch_backward(const sssp_csr &g, int source, const float *dist, const int32_t *pred_edge,
                    const float *grad_dist, float *grad_w, bool validate, sssp_stats *stats,
                    char *ws, int32_t **status_out, hipStream_t st) {
  size_t off = 0;
  auto take = [&](size_t x) {
    char *p = ws + off;
    off += align_up(x ? x : 1, 256);
    return p;
  };
  BwdArgs a;
  a.row_ptr = g.row_ptr;
  a.col = g.col;
  a.dist = dist;
  a.pred_edge = pred_edge;
  a.g = grad_dist;
  a.grad_w = grad_w;
  a.n = g.n;
  a.m = g.m;
  a.source = source;
  a.par = reinterpret_cast<int32_t *>(take(4ull * g.n));
  a.nchild = reinterpret_cast<int32_t *>(take(4ull * g.n));
  a.leaf = reinterpret_cast<int32_t *>(take(4ull * g.n));
  a.mark = reinterpret_cast<int32_t *>(take(4ull * g.n));
  a.acc = reinterpret_cast<double *>(take(8ull * g.n));
  char *misc = take(256);
  a.counts = reinterpret_cast<unsigned long long *>(misc);
  a.status = reinterpret_cast<int32_t *>(misc + 64);
  *status_out = a.status;
  const int work = g.n > g.m ? g.n : g.m;
  int blocks = (work + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
  int vblocks = (g.n + 255) / 256;
  vblocks = vblocks < 1 ? 1 : (vblocks > 4096 ? 4096 : vblocks);
  hipLaunchKernelGGL(k_bwd_init_status, dim3(1), dim3(64), 0, st, a.status, stats);
  if (validate && launch_validate(g, 0, 1, a.status, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_bwd_zero, dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_bwd_parent, dim3(vblocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_bwd_mark, dim3(vblocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_bwd_count, dim3(vblocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_bwd_leaves, dim3(vblocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_bwd_chain, dim3(vblocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_bwd_check, dim3(1), dim3(64), 0, st, a, stats);
  return hipGetLastError() == hipSuccess ? SSSP_OK : SSSP_ERR_HIP;
}

}  // namespace sssp_impl
