// solve.hip -- asynchronous partitioned single-source shortest paths on
// gfx950 (Sec. III-A partitioning, Sec. III-C Alg. 2/3, Sec. III-D
// termination), one persistent launch for one or many solves.
//
// Design, mapped from the paper's MPI processes to one GPU:
//  * A partition (1D vertex block of ceil(n/P) ids) is a scheduling unit.
//    Its inbox is the slice of a per-solve bitmap `dirty` covering its
//    vertices: bit v set = v's label dropped and v awaits expansion.
//  * A workgroup takes an active unit, gathers the unit's dirty vertices that
//    fall in the current delta-bucket (the lowest non-empty one: the local
//    Dijkstra order of Alg. 3 relaxed to buckets), claims them by clearing
//    their bits, and stages them in LDS as a frontier.
//  * It expands the frontier edge-parallel: coalesced CSR streaming, one
//    64-bit atomic min per arc on the head's packed (dist << 32 | edge id)
//    label.  A strictly lower distance sets the head's inbox bit; a head in
//    another unit also raises that unit's active bit -- the asynchronous
//    Bellman-Ford exchange between partitions (send_msg / recv_msgs).
//  * Ctrl::work counts inbox bits plus vertices in flight.  It is raised
//    before work is published and lowered after its consequences are
//    published, so it reaches zero exactly when the global fixed point is
//    reached; that replaces the paper's token-ring / counter termination.
//  * Nothing waits on a particular workgroup: any resident workgroup can
//    take any unit, so the launch needs no co-residency guarantee.  Idle
//    workgroups poll with backoff under a wall-clock limit.
#include "internal.hpp"
#include "launch.hpp"

namespace sssp_impl {

constexpr int FCAP = 2048;  // frontier vertices staged in LDS per batch

template <int WT> struct Dist;
template <> struct Dist<SSSP_W_U32> {
  static constexpr uint32_t INF_BITS = 0xFFFFFFFFu;
  // d + w in 64 bits; overflow when it reaches the unreachable sentinel.
  __device__ static __forceinline__ uint32_t add(uint32_t d, uint32_t w, bool &ovf) {
    unsigned long long s = (unsigned long long)d + w;
    ovf = s >= 0xFFFFFFFFull;
    return (uint32_t)s;
  }
  __device__ static __forceinline__ unsigned long long bucket_end(
      unsigned long long d, unsigned long long delta) {
    if (delta == DELTA_INF) return DELTA_INF;
    return (d / delta + 1) * delta;
  }
};
template <> struct Dist<SSSP_W_F32> {
  static constexpr uint32_t INF_BITS = 0x7F800000u;
  // fl32(d + w), round to nearest even; +inf counts as overflow.
  __device__ static __forceinline__ uint32_t add(uint32_t d, uint32_t w, bool &ovf) {
    float s = __uint_as_float(d) + __uint_as_float(w);
    uint32_t b = __float_as_uint(s);
    ovf = b >= 0x7F800000u;
    return b;
  }
  // End of the bucket [k*delta, (k+1)*delta) holding d, as fp32 bits,
  // rounded up and strictly above d.
  __device__ static __forceinline__ unsigned long long bucket_end(
      unsigned long long d, unsigned long long delta) {
    if (delta == DELTA_INF) return DELTA_INF;
    double df = (double)__uint_as_float((uint32_t)d);
    double dl = (double)__uint_as_float((uint32_t)delta);
    double t = (floor(df / dl) + 1.0) * dl;
    float tf = (float)t;
    if ((double)tf < t) tf = nextafterf(tf, __builtin_inff());
    unsigned long long tb = __float_as_uint(tf);
    if (tb <= d) tb = d + 1;
    return tb;
  }
};

// ------------------------------------------------------------------ setup

// Writes descriptors carried in the kernel arguments into the workspace, so
// a captured launch replays without the host-side tables.
__global__ void k_write_desc(DescChunk c, SolveDesc *table) {
  int i = threadIdx.x;
  if (i < c.count) table[c.first + i] = c.d[i];
}

// Clears the control block, the active-unit bitmap and the stats.
__global__ void k_init_global(SolveArgs a, int nsolves) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int i = t; i < a.nabw; i += stride) a.abits[i] = 0u;
  if (t == 0) {
    a.ctrl->work = nsolves;  // every source starts pending
    a.ctrl->done = 0u;
    a.ctrl->status = 0;
    a.ctrl->nunits = (uint32_t)a.nunits;
  }
  if (a.stats) {
    uint32_t *s = reinterpret_cast<uint32_t *>(a.stats);
    for (int i = t; i < (int)(sizeof(sssp_stats) / 4); i += stride) s[i] = 0u;
  }
}

// Per-solve init (blockIdx.y = solve): labels to +inf, empty inboxes, unit
// tables; the source gets label (0, no edge) and its inbox bit.
__global__ void k_init(SolveArgs a) {
  const int s = blockIdx.y;
  const SolveDesc d = a.desc[s];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int v = t; v < d.n; v += stride)
    d.label[v] = v == d.source ? (unsigned long long)NONE_EDGE : LABEL_INF;
  for (int i = t; i < d.nwords; i += stride)
    d.dirty[i] = i == (d.source >> 5) ? (1u << (d.source & 31)) : 0u;
  for (int p = t; p < d.nparts; p += stride) {
    a.thresh[d.unit0 + p] = d.delta;  // end of bucket 0
    a.unit_solve[d.unit0 + p] = s;
  }
  if (t == 0) {
    const int u = d.unit0 + d.source / d.bsize;
    aor(&a.abits[u >> 5], 1u << (u & 31));
  }
}

// ------------------------------------------------------------------ solve
template <int WT, int BS>
__global__ __launch_bounds__(BS) void k_solve(SolveArgs a) {
  constexpr int EPT = FCAP / BS;  // frontier entries per thread in staging
  constexpr int NW = BS / WAVE;
  static_assert(FCAP % BS == 0, "FCAP must be a multiple of the block size");

  __shared__ int32_t s_v[FCAP];      // claimed vertex, or -1 for a hole
  __shared__ uint32_t s_d[FCAP];     // its distance bits at expansion time
  __shared__ int32_t s_rs[FCAP];     // its first edge
  __shared__ int32_t s_off[FCAP + 1];// exclusive prefix of degrees
  __shared__ int s_ws[NW + 1];
  __shared__ SolveDesc s_desc;
  __shared__ int s_unit, s_solve, s_cnt, s_left, s_push, s_exit, s_claimed;
  __shared__ unsigned long long s_min;
  __shared__ unsigned int s_upd, s_cross, s_new;

  const int tid = threadIdx.x;
  Ctrl *ctrl = a.ctrl;
  if (tid == 0) {
    s_exit = ld_rlx(&ctrl->status) != 0;
    s_solve = -1;
  }
  __syncthreads();
  if (s_exit) return;

  const unsigned long long t_start = wall_clock64();
  const int start_word = (int)((blockIdx.x * 2654435761u) % (unsigned)a.nabw);
  int rounds = 0;
  int stay = -1;

  for (;;) {
    // ---------------------------------------------------------- pick a unit
    if (tid == 0) {
      s_unit = -1;
      if (ld_rlx(&ctrl->done)) {
        s_exit = 1;
      } else if (a.time_limit && wall_clock64() - t_start > a.time_limit) {
        set_status(&ctrl->status, SSSP_ERR_TIMEOUT);
        st_rlx(&ctrl->done, 1u);
        s_exit = 1;
      }
    }
    __syncthreads();
    if (s_exit) break;

    int unit = stay;
    if (unit < 0) {
      for (int base = 0; base < a.nabw; base += BS) {
        const int i = base + tid;
        int found = 0x7FFFFFFF;
        if (i < a.nabw) {
          int wi = start_word + i;
          if (wi >= a.nabw) wi -= a.nabw;
          if (ld_rlx(&a.abits[wi])) found = i;
        }
        found = wave_min(found);
        if (lane_id() == 0) s_ws[tid / WAVE] = found;
        __syncthreads();
        if (tid == 0) {
          int mn = 0x7FFFFFFF;
          for (int k = 0; k < NW; k++) mn = s_ws[k] < mn ? s_ws[k] : mn;
          if (mn != 0x7FFFFFFF) {
            int wi = start_word + mn;
            if (wi >= a.nabw) wi -= a.nabw;
            uint32_t bits = ld_rlx(&a.abits[wi]);
            const int r = blockIdx.x & 31;
            while (bits) {
              // rotate the pick by block id to spread workgroups over units
              uint32_t rot = (bits >> r) | (bits << ((32 - r) & 31));
              int b = (__ffs(rot) - 1 + r) & 31;
              uint32_t mb = 1u << b;
              uint32_t old = aand_acq(&a.abits[wi], ~mb);
              if (old & mb) {
                s_unit = wi * 32 + b;
                break;
              }
              bits = old & ~mb;
            }
          }
          s_ws[NW] = mn;
        }
        __syncthreads();
        const int mn = s_ws[NW];
        __syncthreads();
        if (mn != 0x7FFFFFFF) break;
      }
      unit = s_unit;
    }

    if (unit < 0) {
      // idle: finished when no work is pending anywhere
      if (tid == 0) {
        if (ld_rlx(&ctrl->work) <= 0) {
          st_rlx(&ctrl->done, 1u);
          s_exit = 1;
        }
      }
      __syncthreads();
      if (s_exit) break;
      __builtin_amdgcn_s_sleep(16);
      continue;
    }

    // ------------------------------------------------- unit -> descriptor
    if (tid == 0) {
      const int sv = a.unit_solve[unit];
      if (sv != s_solve) {
        s_solve = sv;
        s_desc = a.desc[sv];
      }
    }
    __syncthreads();
    const int n = s_desc.n;
    const int m = s_desc.m;
    const int bsize = s_desc.bsize;
    const int source = s_desc.source;
    const int unit0 = s_desc.unit0;
    const unsigned long long delta = s_desc.delta;
    const int32_t *__restrict__ row_ptr = s_desc.row_ptr;
    const int32_t *__restrict__ col = s_desc.col;
    const uint32_t *__restrict__ wgt = s_desc.w;
    unsigned long long *label = s_desc.label;
    uint32_t *dirty = s_desc.dirty;

    const int part = unit - unit0;
    const int vlo = part * bsize;
    const int vhi = min(n, vlo + bsize);
    const int wlo = vlo >> 5;
    const int whi = (vhi - 1) >> 5;

    // ------------------------------ gather + claim the lowest bucket (<= 2 tries)
    unsigned long long T = ld_rlx(&a.thresh[unit]);
    int cnt = 0;
    for (int attempt = 0; attempt < 2; attempt++) {
      if (tid == 0) {
        s_cnt = 0;
        s_left = 0;
        s_min = ~0ull;
        s_claimed = 0;
      }
      __syncthreads();
      for (int wi = wlo + tid; wi <= whi; wi += BS) {
        uint32_t mask = ~0u;
        if (wi == wlo) mask &= ~0u << (vlo & 31);
        if (wi == whi) {
          const int hb = (vhi - 1) & 31;
          mask &= hb == 31 ? ~0u : ((1u << (hb + 1)) - 1u);
        }
        const uint32_t bits = ld_rlx(&dirty[wi]) & mask;
        if (!bits) continue;
        uint32_t near = 0;
        unsigned long long mn = ~0ull;
        for (uint32_t b = bits; b; b &= b - 1) {
          const int k = __ffs(b) - 1;
          const unsigned long long dv = ld_rlx(&label[wi * 32 + k]) >> 32;
          if (dv < T) near |= 1u << k;
          else mn = dv < mn ? dv : mn;
        }
        if (near) {
          const int c = __popc(near);
          const int base = atomicAdd(&s_cnt, c);
          if (base >= FCAP) {
            near = 0;
          } else if (base + c > FCAP) {
            uint32_t keep = 0, t = near;
            for (int j = 0; j < FCAP - base; j++) {
              keep |= t & (~t + 1u);
              t &= t - 1;
            }
            near = keep;
          }
          if (near) {
            const uint32_t got = aand_acq(&dirty[wi], ~near) & near;
            int j = base;
            for (uint32_t b = near; b; b &= b - 1) {
              const int k = __ffs(b) - 1;
              s_v[j++] = (got >> k) & 1u ? wi * 32 + k : -1;
            }
          }
        }
        if (bits & ~near) s_left = 1;
        if (mn != ~0ull) atomicMin(&s_min, mn);
      }
      __syncthreads();
      cnt = min(s_cnt, FCAP);
      const unsigned long long smin = s_min;
      if (cnt > 0 || smin == ~0ull) break;
      // nothing in the current bucket but later ones are not empty: open the
      // lowest non-empty bucket
      T = Dist<WT>::bucket_end(smin, delta);
      if (tid == 0) amax(&a.thresh[unit], T);
      __syncthreads();
    }
    if (tid == 0 && s_left) aor(&a.abits[unit >> 5], 1u << (unit & 31));
    if (cnt == 0) {
      stay = -1;
      __syncthreads();
      continue;
    }

    // ------------------------------------------ stage rows of the frontier
    int degs[EPT];
    int lsum = 0, nclaim = 0;
#pragma unroll
    for (int j = 0; j < EPT; j++) {
      const int k = tid * EPT + j;
      int deg = 0;
      if (k < cnt) {
        const int u = s_v[k];
        int rs = 0;
        if (u >= 0) {
          nclaim++;
          const unsigned long long lab = ld_rlx(&label[u]);
          s_d[k] = (uint32_t)(lab >> 32);
          rs = row_ptr[u];
          int re = row_ptr[u + 1];
          if (rs < 0 || re < rs || re > m) {
            set_status(&ctrl->status, SSSP_ERR_CSR);
            rs = 0;
            re = 0;
          }
          deg = re - rs;
        }
        s_rs[k] = rs;
      }
      degs[j] = deg;
      lsum += deg;
    }
    nclaim = wave_sum(nclaim);
    if (lane_id() == 0 && nclaim) atomicAdd(&s_claimed, nclaim);
    int tot;
    int run = block_excl_scan<BS>(lsum, s_ws, &tot);
#pragma unroll
    for (int j = 0; j < EPT; j++) {
      const int k = tid * EPT + j;
      if (k < cnt) s_off[k] = run;
      run += degs[j];
    }
    if (tid == 0) {
      s_off[cnt] = tot;
      // raise the pending count by an upper bound of the inbox bits this
      // batch can set, before any of them is published
      if (tot) aadd(&ctrl->work, (long long)tot);
      s_upd = 0;
      s_cross = 0;
      s_new = 0;
      s_push = 0;
    }
    __syncthreads();

    // ---------------------------------------------- edge-parallel relaxation
    unsigned int upd = 0, cross = 0, nnew = 0;
    int push = 0;
    for (int idx = tid; idx < tot; idx += BS) {
      int lo = 0, hi = cnt - 1;  // last k with s_off[k] <= idx
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= idx) lo = mid;
        else hi = mid - 1;
      }
      const int e = s_rs[lo] + (idx - s_off[lo]);
      const int v = col[e];
      const uint32_t wv = wgt[e];
      if ((unsigned)v >= (unsigned)n) {
        set_status(&ctrl->status, SSSP_ERR_CSR);
        continue;
      }
      if (v == source) continue;
      bool ovf;
      const uint32_t nd = Dist<WT>::add(s_d[lo], wv, ovf);
      if (ovf) {
        set_status(&ctrl->status, SSSP_ERR_OVERFLOW);
        continue;
      }
      const unsigned long long packed = ((unsigned long long)nd << 32) | (uint32_t)e;
      if (packed >= ld_rlx(&label[v])) continue;
      const unsigned long long old = amin(&label[v], packed);
      if ((uint32_t)(old >> 32) <= nd) continue;  // distance not lowered
      upd++;
      const int q = v / bsize;
      if (q != part) cross++;
      const uint32_t bit = 1u << (v & 31);
      if (aor(&dirty[v >> 5], bit) & bit) continue;  // already pending
      nnew++;
      if (q != part) {
        const int gu = unit0 + q;
        const uint32_t ab = 1u << (gu & 31);
        if (!(ld_rlx(&a.abits[gu >> 5]) & ab)) aor(&a.abits[gu >> 5], ab);
      } else {
        push = 1;
      }
    }
    upd = wave_sum(upd);
    cross = wave_sum(cross);
    nnew = wave_sum(nnew);
    if (lane_id() == 0) {
      if (upd) atomicAdd(&s_upd, upd);
      if (cross) atomicAdd(&s_cross, cross);
      if (nnew) atomicAdd(&s_new, nnew);
    }
    if (push) s_push = 1;
    __syncthreads();
    if (tid == 0) {
      // every consequence of this batch is published: settle the count
      aadd(&ctrl->work, (long long)s_new - (long long)tot - (long long)s_claimed);
      if (a.stats) {
        stat_add(&a.stats->edges_relaxed, (uint64_t)tot);
        stat_add(&a.stats->label_updates, (uint64_t)s_upd);
        stat_add(&a.stats->cross_updates, (uint64_t)s_cross);
        stat_add(&a.stats->vertices_expanded, (uint64_t)s_claimed);
        stat_add(&a.stats->batches, 1);
      }
      if (a.max_rounds > 0 && ++rounds >= a.max_rounds) {
        set_status(&ctrl->status, SSSP_ERR_TIMEOUT);
        st_rlx(&ctrl->done, 1u);
      }
    }
    stay = s_push ? unit : -1;
    __syncthreads();
  }
}

// --------------------------------------------------------------- epilogue
// Unpacks labels: dist = high word (sentinel kept), pred_edge = low word
// (-1 for none), pred = tail of pred_edge by binary search in row_ptr.
template <int WT>
__global__ void k_epilogue(SolveArgs a) {
  const int s = blockIdx.y;
  const SolveDesc d = a.desc[s];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  uint32_t *dist = static_cast<uint32_t *>(d.dist);
  for (int v = t; v < d.n; v += stride) {
    const unsigned long long lab = d.label[v];
    uint32_t dv;
    int32_t pe = -1, pv = -1;
    if (lab == LABEL_INF) {
      dv = Dist<WT>::INF_BITS;
    } else {
      dv = (uint32_t)(lab >> 32);
      const uint32_t lo = (uint32_t)lab;
      if (lo != NONE_EDGE) {
        pe = (int32_t)lo;
        if (d.pred) {
          int l = 0, h = d.n - 1;  // largest u with row_ptr[u] <= pe
          while (l < h) {
            const int mid = l + ((h - l + 1) >> 1);
            if (d.row_ptr[mid] <= pe) l = mid;
            else h = mid - 1;
          }
          pv = l;
        }
      }
    }
    dist[v] = dv;
    if (d.pred) d.pred[v] = pv;
    if (d.pred_edge) d.pred_edge[v] = pe;
  }
  if (s == 0 && t == 0 && a.stats) {
    a.stats->status = a.ctrl->status;
    a.stats->num_partitions = d.nparts;
    a.stats->delta_bits = d.delta;
  }
}

// ------------------------------------------------------------- validation
// CSR and weight checks; the first violation is written to *status.
__global__ void k_validate(const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                           int n, int m, int wtype, int need_sorted, int need_positive,
                           int32_t *status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  if (t == 0 && (row_ptr[0] != 0 || row_ptr[n] != m)) set_status(status, SSSP_ERR_CSR);
  for (int u = t; u < n; u += stride) {
    const int a = row_ptr[u], b = row_ptr[u + 1];
    if (a > b || a < 0 || b > m) {
      set_status(status, SSSP_ERR_CSR);
      continue;
    }
    if (need_sorted)
      for (int e = a + 1; e < b; e++)
        if (col[e] < col[e - 1]) {
          set_status(status, SSSP_ERR_UNSORTED);
          break;
        }
  }
  for (int e = t; e < m; e += stride) {
    if ((unsigned)col[e] >= (unsigned)n) set_status(status, SSSP_ERR_CSR);
    const uint32_t x = w[e];
    if (wtype == SSSP_W_F32) {
      if ((x >> 31) || (x & 0x7F800000u) == 0x7F800000u) set_status(status, SSSP_ERR_WEIGHT);
      else if (need_positive && x == 0u) set_status(status, SSSP_ERR_ZERO_WEIGHT);
    } else if (need_positive && x == 0u) {
      set_status(status, SSSP_ERR_ZERO_WEIGHT);
    }
  }
}

__global__ void k_copy_status(const int32_t *status, sssp_stats *stats) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && stats) stats->status = *status;
}

// ------------------------------------------------------------ host launch
hipError_t launch_validate(const sssp_csr &g, int need_sorted, int need_positive,
                           int32_t *status, hipStream_t st) {
  const int work = g.n > g.m ? g.n : g.m;
  int blocks = (work + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
  hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, st, g.row_ptr, g.col,
                     static_cast<const uint32_t *>(g.w), g.n, g.m, g.wtype, need_sorted,
                     need_positive, status);
  return hipGetLastError();
}

hipError_t launch_write_desc(const DescChunk &c, SolveDesc *table, hipStream_t st) {
  hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(32), 0, st, c, table);
  return hipGetLastError();
}

hipError_t launch_init(const SolveArgs &a, int nsolves, int max_n, hipStream_t st) {
  int gb = (a.nabw + 255) / 256;
  gb = gb < 1 ? 1 : (gb > 256 ? 256 : gb);
  hipLaunchKernelGGL(k_init_global, dim3(gb), dim3(256), 0, st, a, nsolves);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int bx = (max_n + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 1024 ? 1024 : bx);
  hipLaunchKernelGGL(k_init, dim3(bx, nsolves), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int WT, int BS>
static hipError_t launch_solve_t(const SolveArgs &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_solve<WT, BS>), dim3(grid), dim3(BS), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs &a, int wtype, int bs, int grid, hipStream_t st) {
  if (wtype == SSSP_W_U32) {
    if (bs == 256) return launch_solve_t<SSSP_W_U32, 256>(a, grid, st);
    if (bs == 512) return launch_solve_t<SSSP_W_U32, 512>(a, grid, st);
    return launch_solve_t<SSSP_W_U32, 1024>(a, grid, st);
  }
  if (bs == 256) return launch_solve_t<SSSP_W_F32, 256>(a, grid, st);
  if (bs == 512) return launch_solve_t<SSSP_W_F32, 512>(a, grid, st);
  return launch_solve_t<SSSP_W_F32, 1024>(a, grid, st);
}

int solve_max_blocks_per_cu(int wtype, int bs) {
  int nb = 0;
  hipError_t e;
#define SSSP_OCC(WT, BS)                                                                   \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_solve<WT, BS>, BS, 0);
  if (wtype == SSSP_W_U32) {
    if (bs == 256) { SSSP_OCC(SSSP_W_U32, 256) }
    else if (bs == 512) { SSSP_OCC(SSSP_W_U32, 512) }
    else { SSSP_OCC(SSSP_W_U32, 1024) }
  } else {
    if (bs == 256) { SSSP_OCC(SSSP_W_F32, 256) }
    else if (bs == 512) { SSSP_OCC(SSSP_W_F32, 512) }
    else { SSSP_OCC(SSSP_W_F32, 1024) }
  }
#undef SSSP_OCC
  return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_epilogue(const SolveArgs &a, int wtype, int nsolves, int max_n,
                           hipStream_t st) {
  int bx = (max_n + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 1024 ? 1024 : bx);
  if (wtype == SSSP_W_U32)
    hipLaunchKernelGGL(k_epilogue<SSSP_W_U32>, dim3(bx, nsolves), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_epilogue<SSSP_W_F32>, dim3(bx, nsolves), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace sssp_impl
