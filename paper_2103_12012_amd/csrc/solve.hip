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
//    another unit also wakes that unit (its pending minimum and active bit,
//    gathered per unit in LDS and published once per round or batch) --
//    the asynchronous Bellman-Ford exchange between partitions (send_msg /
//    recv_msgs).
//  * Ctrl::work counts inbox bits plus vertices in flight.  It is raised
//    before work is published and lowered after its consequences are
//    published, so it reaches zero exactly when the global fixed point is
//    reached; that replaces the paper's token-ring / counter termination.
//  * Nothing waits on a particular workgroup: any resident workgroup can
//    take any unit, so the launch needs no co-residency guarantee.  Idle
//    workgroups poll with backoff under a wall-clock limit.
#include <climits>

#include "internal.hpp"
#include "launch.hpp"

namespace sssp_impl {

constexpr int FCAP = 1024;  // frontier vertices staged in LDS per round
constexpr int MAXB = 65536; // largest partition (vertices): LDS dedupe bitmap and gather mask
constexpr int ACT_SLOTS = 512;  // deferred unit activations per batch (LDS hash)
constexpr int ACT_FEW = 32;     // at most this many units recorded: wake them every round

// Activating the unit a push lands in (its pending minimum and active bit)
// is deferred: the pushes of a batch are gathered per destination unit in
// an LDS table, and each unit is published once.  With at most ACT_FEW
// units recorded (a thin frontier crossing into a neighbour, where waking
// it soon is the critical path) the table is published at the end of every
// round, otherwise at the end of the batch, before the batch's pending-work
// surplus is returned.  One atomic min and one atomic or per unit replace
// one of each per cross-partition push, which all workgroups aimed at the
// same few hundred words.
//
// Records a push into unit gu at distance d; false when the table is
// crowded (the caller activates directly).
__device__ __forceinline__ bool act_defer(int32_t *keys, uint32_t *dmin, int *nrec, int gu, uint32_t d) {
  uint32_t h = ((uint32_t)gu * 2654435761u) >> 23;  // 512 slots
  for (int probe = 0; probe < 8; probe++) {
    const int old = atomicCAS(&keys[h], -1, gu);
    if (old == -1) atomicAdd(nrec, 1);
    if (old == -1 || old == gu) {
      atomicMin(&dmin[h], d);
      return true;
    }
    h = (h + 1) & (ACT_SLOTS - 1);
  }
  return false;
}
// Buffered cross-partition updates (solve mode SOLVE_BUFFERED): a candidate
// label for a head in another partition is not applied at once; the batch
// keeps the least candidate per head in an LDS table and applies each
// distinct head once, with one atomic min.  Push-out criteria: the end of a
// settle round once the table holds SSSP_XB_FLUSH heads (default 1: every
// round that buffered anything; flushing only at half a table was slower,
// grid 4096^2 79 against 69 ms), a full table (a candidate that finds no
// slot goes straight to HBM), and the end of the batch, before the batch's
// pending work is returned, so nothing buffered is ever invisible to
// termination.  Arcs of one round that lead into the same head thus cost
// one global atomic instead of one each: the paper's message buffering,
// with min-combining.
constexpr int XB_SLOTS = 1024;
#ifndef SSSP_XB_FLUSH
#define SSSP_XB_FLUSH 1
#endif

// Keeps the least packed candidate pk for head v; false when the table is
// crowded (the caller applies the candidate directly).
__device__ __forceinline__ bool xb_insert(int32_t *keys, unsigned long long *vals, int *nrec,
                                          int v, unsigned long long pk) {
  uint32_t h = ((uint32_t)v * 2654435761u) >> 22;  // 1024 slots
  for (int probe = 0; probe < 8; probe++) {
    const int old = atomicCAS(&keys[h], -1, v);
    if (old == -1) atomicAdd(nrec, 1);
    if (old == -1 || old == v) {
      atomicMin(&vals[h], pk);
      return true;
    }
    h = (h + 1) & (XB_SLOTS - 1);
  }
  return false;
}

constexpr int MAX_ROUNDS_PER_BATCH = 256;

// Idle-time pruning (SOLVE_IDLE_PRUNE, Sec. III-B: processes without
// messages use their idle time for Trishla).  A workgroup that finds no
// active unit takes a ticket for PRUNE_CHUNK consecutive vertices and tests
// every arc (u, x, W) of each: deleted when a middle vertex y of u's own
// partition (LOCAL scope), y != u and y != x, has arcs (u, y, w1) and
// (y, x, w2) with w1 + w2 < W.  The heads of u go into an LDS hash table;
// the rows of u's middles are walked edge-parallel and every two-arc cost
// is min-combined into its head's slot; then each arc of u is compared
// with its head's least detour.  Rows with more than PT_SLOTS / 2 arcs or
// more than PRUNE_MAX_WEDGES two-arc paths are left alone, which keeps a
// ticket short: any subset of the LOCAL deletion set is a valid result
// (a deleted arc is never tight, so distances and predecessors do not
// change), and the solve ends as soon as no work is pending, whether or
// not every ticket was taken.
constexpr int PT_SLOTS = 2048;
constexpr int PRUNE_MAX_WEDGES = 1 << 16;

__device__ __forceinline__ uint32_t pt_hash(int x) { return ((uint32_t)x * 2654435761u) >> 21; }

// Slot of key x in the table (inserted if absent); the table never fills
// (at most PT_SLOTS / 2 keys).
__device__ __forceinline__ int pt_insert(int32_t *keys, int x) {
  uint32_t h = pt_hash(x);
  for (int probe = 0; probe < PT_SLOTS; probe++) {
    const int old = atomicCAS(&keys[h], -1, x);
    if (old == -1 || old == x) return (int)h;
    h = (h + 1) & (PT_SLOTS - 1);
  }
  return -1;
}
__device__ __forceinline__ int pt_find(const int32_t *keys, int x) {
  uint32_t h = pt_hash(x);
  for (int probe = 0; probe < PT_SLOTS; probe++) {
    const int k = keys[h];
    if (k == x) return (int)h;
    if (k == -1) return -1;
    h = (h + 1) & (PT_SLOTS - 1);
  }
  return -1;
}
// Two-arc cost in a form that orders like the real sum: the integer sum, or
// the double sum of two fp32 costs (as bits: nonnegative doubles order like
// their bit patterns).  The double sum is exact unless the costs are more
// than 29 binary orders apart, and then the rounding cannot change its
// comparison with an fp32 cost.
template <int WT>
__device__ __forceinline__ unsigned long long pair_cost(uint32_t w1, uint32_t w2) {
  if (WT == SSSP_W_U32) return (unsigned long long)w1 + w2;
  const double d = (double)__uint_as_float(w1) + (double)__uint_as_float(w2);
  return (unsigned long long)__double_as_longlong(d);
}
template <int WT>
__device__ __forceinline__ bool pair_beats(unsigned long long c, uint32_t W) {
  if (c == ~0ull) return false;
  if (WT == SSSP_W_U32) return c < (unsigned long long)W;
  return __longlong_as_double((long long)c) < (double)__uint_as_float(W);
}

// Binary min-heap in LDS for the heap mode (one thread operates on it):
// the root is the least key; children of i are 2i+1 and 2i+2.
constexpr int HCAP = 2048;
__device__ __forceinline__ void heap_down(unsigned long long *h, int n, int i) {
  const unsigned long long x = h[i];
  for (;;) {
    int c = 2 * i + 1;
    if (c >= n) break;
    unsigned long long cv = h[c];
    if (c + 1 < n && h[c + 1] < cv) {
      c++;
      cv = h[c];
    }
    if (x <= cv) break;
    h[i] = cv;
    i = c;
  }
  h[i] = x;
}
// Places key x at position i (the new last slot) and restores heap order.
__device__ __forceinline__ void heap_up(unsigned long long *h, int i, unsigned long long x) {
  while (i > 0) {
    const int p = (i - 1) >> 1;
    const unsigned long long pv = h[p];
    if (pv <= x) break;
    h[i] = pv;
    i = p;
  }
  h[i] = x;
}
// Pending-count raise of one batch: above MAX_ROUNDS_PER_BATCH * (2^31 - 1)
// inbox bits, and 2^50 per workgroup keeps the sum far from overflow.
constexpr long long RAISE = 1ll << 50;
static_assert((long long)MAX_ROUNDS_PER_BATCH * 0x7FFFFFFFll < RAISE, "raise too small");

template <int WT> struct Dist;
template <> struct Dist<SSSP_W_U32> {
  static constexpr uint32_t INF_BITS = 0xFFFFFFFFu;
  // d <= g + window
  __device__ static __forceinline__ bool within(unsigned long long d, unsigned long long g,
                                                unsigned long long window) {
    return d <= g + window;
  }
  // d + w in 64 bits; a sum reaching the unreachable sentinel does not fit.
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
  // d <= g + window, on the fp32 values (saturated keys count as +inf)
  __device__ static __forceinline__ bool within(unsigned long long d, unsigned long long g,
                                                unsigned long long window) {
    if (d >= 0x7F800000ull) return false;
    return __uint_as_float((uint32_t)d) <=
           __uint_as_float((uint32_t)g) + __uint_as_float((uint32_t)window);
  }
  // fl32(d + w), round to nearest even; +inf does not fit.
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
// Word of the active-unit bitmap holding unit u, and u's bit in it: each word
// holds 8 units and sits on a 128-byte line of its own (ABW_STRIDE words
// apart), since every wakeup and every claim of a unit is an atomic on that
// word; fewer units per line means less contention (32 per word: 10% slower
// on R-MAT 20), and the pick still reads one word per 8 units.
__device__ __forceinline__ int abw(int u) { return (u / ABW_UNITS) * ABW_STRIDE; }
__device__ __forceinline__ uint32_t abit(int u) { return 1u << (u % ABW_UNITS); }


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
  for (int i = t; i < a.nabw; i += stride) a.abits[i * ABW_STRIDE] = 0u;
  if (t == 0) {
    a.ctrl->work = nsolves;  // every source starts pending
    a.ctrl->done = 0u;
    a.ctrl->status = 0;
    a.ctrl->nunits = (uint32_t)a.nunits;
    a.ctrl->ovf = 0u;
    a.ctrl->prune_next = 0;
    a.ctrl->window = a.window;
  }
  if (a.stats) {
    uint32_t *s = reinterpret_cast<uint32_t *>(a.stats);
    for (int i = t; i < (int)(sizeof(sssp_stats) / 4); i += stride) s[i] = 0u;
  }
  if (a.keepbits) {  // every arc starts kept
    const int words = (a.desc_m0 + 31) / 32;
    for (int i = t; i < words; i += stride) a.keepbits[i] = ~0u;
  }
}

// Copies the keep bits of an idle-pruning solve to the caller's uint8 flags.
__global__ void k_keep_out(SolveArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < a.desc_m0; e += stride) a.keep_out[e] = (a.keepbits[e >> 5] >> (e & 31)) & 1u;
}

// Per-solve init (blockIdx.y = solve): labels to +inf, empty inboxes, unit
// tables; the source gets label (0, no edge) and its inbox bit, and its unit
// the pending minimum 0.
__global__ void k_init(SolveArgs a) {
  const int s = blockIdx.y;
  const SolveDesc d = a.desc[s];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  const int ps = d.source / d.bsize;
  for (int v = t; v < d.n; v += stride)
    d.label[v] = v == d.source ? (unsigned long long)NONE_EDGE : LABEL_INF;
  for (int i = t; i < d.nwords; i += stride)
    d.dirty[i] = i == (d.source >> 5) ? (1u << (d.source & 31)) : 0u;
  for (int p = t; p < d.nparts; p += stride) {
    a.unit_min[d.unit0 + p] = p == ps ? 0ull : LABEL_INF;
    a.unit_solve[d.unit0 + p] = s;
  }
  if (t == 0) {
    const int u = d.unit0 + ps;
    aor(&a.abits[abw(u)], abit(u));
  }
}

// Bucket width of every solve left automatic (one workgroup per solve):
// auto_factor times the mean of up to 4096 arc costs sampled at a fixed
// stride; a single solve's lag window follows from it.
template <int WT>
__global__ __launch_bounds__(256) void k_auto_delta(SolveArgs a) {
  __shared__ double s_part[256 / WAVE];
  SolveDesc *dd = const_cast<SolveDesc *>(a.desc) + blockIdx.x;
  if (dd->delta != DELTA_AUTO) return;
  const int m = dd->m;
  const int k = m < 4096 ? m : 4096;
  double acc = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const uint32_t w = dd->w[(long long)i * m / k];
    acc += WT == SSSP_W_U32 ? (double)w : (double)__uint_as_float(w);
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, WAVE);
  if (lane_id() == 0) s_part[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double sum = 0.0;
  for (int i = 0; i < 256 / WAVE; i++) sum += s_part[i];
  const double width = (double)dd->auto_factor * (k > 0 ? sum / k : 1.0);
  unsigned long long delta, window = DELTA_INF;
  if (WT == SSSP_W_U32) {
    const double c = ceil(width);
    delta = c < 1.0 ? 1ull : (c >= 4294967296.0 ? DELTA_INF : (unsigned long long)c);
    if (a.auto_lag > 0 && delta != DELTA_INF) window = delta * (unsigned long long)a.auto_lag;
  } else {
    float f = (float)width;
    if (!(f > 0.0f)) f = 1.17549435e-38f;  // smallest normal
    delta = f == __builtin_inff() ? DELTA_INF : __float_as_uint(f);
    if (a.auto_lag > 0 && delta != DELTA_INF) window = __float_as_uint(f * (float)a.auto_lag);
  }
  dd->delta = delta;
  if (a.num_solves == 1) a.ctrl->window = window;
}

// Bijective 32-bit mix of a unit id (per-workgroup key) used to break ties
// between units of equal pending minimum differently in every workgroup.
__device__ __forceinline__ uint32_t unit_mix(uint32_t u, uint32_t key) {
  return (u ^ key) * 0x9E3779B1u;
}
__device__ __forceinline__ uint32_t unit_unmix(uint32_t x, uint32_t key) {
  return (x * 0x0E8B2F51u) ^ key;
}

// Applies every buffered cross-partition candidate (one atomic min per
// distinct head), marks lowered heads in their owners' inboxes and records
// the owners' wakeups; clears the table.  Called by the whole workgroup
// after a barrier; the caller reduces the counters and clears the count.
template <int BS>
__device__ __forceinline__ void xb_flush(int32_t *keys, unsigned long long *vals,
                                         unsigned long long *label, uint32_t *dirty, int bsize,
                                         int unit0, unsigned long long *unit_min, uint32_t *abits,
                                         int32_t *actk, uint32_t *actd, int *actn,
                                         unsigned int &upd, unsigned int &cross,
                                         unsigned int &nnew) {
  constexpr int K = XB_SLOTS / BS < 4 ? (XB_SLOTS / BS > 0 ? XB_SLOTS / BS : 1) : 4;
  for (int i0 = 0; i0 < XB_SLOTS; i0 += BS * K) {
    int v[K];
    unsigned long long pk[K], cur[K];
#pragma unroll
    for (int j = 0; j < K; j++) {
      const int i = i0 + j * BS + (int)threadIdx.x;
      v[j] = i < XB_SLOTS ? keys[i] : -1;
      if (v[j] >= 0) {
        pk[j] = vals[i];
        keys[i] = -1;
        vals[i] = ~0ull;
        cur[j] = ld_rlx(&label[v[j]]);
      }
    }
#pragma unroll
    for (int j = 0; j < K; j++) {
      if (v[j] >= 0 && pk[j] < cur[j]) cur[j] = amin(&label[v[j]], pk[j]);
      else v[j] = -1;
    }
    uint32_t ob[K];
#pragma unroll
    for (int j = 0; j < K; j++) {
      if (v[j] < 0) continue;
      if ((uint32_t)(cur[j] >> 32) <= (uint32_t)(pk[j] >> 32)) {
        v[j] = -1;
        continue;
      }
      upd++;
      cross++;
      ob[j] = aor(&dirty[v[j] >> 5], 1u << (v[j] & 31));
    }
#pragma unroll
    for (int j = 0; j < K; j++) {
      if (v[j] < 0 || ((ob[j] >> (v[j] & 31)) & 1u)) continue;  // already pending
      nnew++;
      const int gu = unit0 + v[j] / bsize;
      const uint32_t nd = (uint32_t)(pk[j] >> 32);
      if (!act_defer(actk, actd, actn, gu, nd)) {
        amin(&unit_min[gu], (unsigned long long)nd);
        aor(&abits[abw(gu)], abit(gu));
      }
    }
  }
}

// ------------------------------------------------------------------ solve
//
// One batch of a workgroup:
//  1. pick: among active units, the one with the least pending minimum
//     (best-first over partitions), skipping units more than `window` above
//     the global least (bounded lag); claim it by clearing its active bit;
//  2. gather: list the unit's inbox bits (up to FCAP) and load their labels
//     in parallel; the lowest non-empty bucket [kD, (k+1)D) of the listed
//     distances is claimed, one atomic and-not per inbox word;
//  3. stage the claimed vertices' rows and distances in LDS and scan the
//     degrees;
//  4. relax edge-parallel, U arcs per thread in flight;
//  5. settle the pending count, publish the unit's remaining minimum and
//     reactivate it if it still holds work.
#ifndef SSSP_SOLVE_MIN_WAVES
#define SSSP_SOLVE_MIN_WAVES 2
#endif
template <int WT, int BS, int MODE>
__global__ __launch_bounds__(BS, BS == 1024 ? 4 : SSSP_SOLVE_MIN_WAVES) void k_solve(SolveArgs a) {
  constexpr int NW = BS / WAVE;
  constexpr int U = 4;  // arcs per thread per round
  constexpr int EPT = FCAP / BS;
  constexpr bool XBUF = MODE == SOLVE_BUFFERED;
  constexpr bool HEAP = MODE == SOLVE_HEAP;
  constexpr bool IPRUNE = MODE == SOLVE_IDLE_PRUNE;
  static_assert(FCAP % BS == 0, "FCAP must be a multiple of the block size");

  __shared__ int32_t s_v[FCAP];       // claimed frontier vertices
  __shared__ uint32_t s_vd[FCAP];     // their distances (round 0)
  __shared__ uint32_t s_d[FCAP];      // gather: listed distances; relax: frontier distances
  __shared__ int32_t s_rs[FCAP];      // gather: listed vertices;  relax: first arc of each
  __shared__ int32_t s_off[FCAP + 1]; // relax: degree prefix
  __shared__ uint32_t s_fm[MAXB / 32 + 1];  // gather: far mask per inbox word (a block
                                            // not starting on a word spans one more)
  __shared__ int s_ws[NW + 1];
  __shared__ unsigned long long s_red[NW];
  __shared__ SolveDesc s_desc;
  __shared__ int s_unit, s_solve, s_exit, s_nlist, s_cnt, s_idle, s_stay;
  __shared__ unsigned long long s_far, s_lmin, s_gmin;
  __shared__ unsigned int s_upd, s_cross, s_new;
  __shared__ int32_t s_nv[FCAP];           // next round's frontier (same bucket)
  __shared__ uint32_t s_mark[MAXB / 32];   // partition-local dedupe of s_nv
  __shared__ int s_ncnt;
  __shared__ long long s_tot, s_exp;
  __shared__ int32_t s_actk[ACT_SLOTS];   // deferred activations: unit (-1 = free)
  __shared__ uint32_t s_actd[ACT_SLOTS];  //   and the least distance pushed into it
  __shared__ int s_actn;                  //   units recorded
  __shared__ int32_t s_xbk[XBUF ? XB_SLOTS : 1];             // buffered heads (-1 = free)
  __shared__ unsigned long long s_xbv[XBUF ? XB_SLOTS : 1];  //   least candidate label
  __shared__ int s_xbn;                                      //   heads buffered
  __shared__ unsigned long long s_heap[HEAP ? HCAP : 1];     // heap mode: (dist, vertex) keys
  __shared__ int s_hn, s_hu, s_hr0, s_hr1;                   //   size; popped vertex and row
  __shared__ uint32_t s_hdu;                                 //   its distance
  __shared__ int32_t s_pk[IPRUNE ? PT_SLOTS : 1];            // idle prune: heads of u
  __shared__ unsigned long long s_pc[IPRUNE ? PT_SLOTS : 1]; //   least detour per head
  __shared__ int s_ptask, s_pm;                              //   ticket; middles staged
  __shared__ unsigned long long s_pruned, s_wedges;          //   arcs deleted; paths examined

  const int tid0 = threadIdx.x;
  if constexpr (XBUF) {
    for (int i = tid0; i < XB_SLOTS; i += BS) {
      s_xbk[i] = -1;
      s_xbv[i] = ~0ull;
    }
    if (tid0 == 0) s_xbn = 0;
  }
  for (int i = tid0; i < MAXB / 32; i += BS) s_mark[i] = 0u;
  for (int i = tid0; i < ACT_SLOTS; i += BS) {
    s_actk[i] = -1;
    s_actd[i] = 0xFFFFFFFFu;
  }
  if (tid0 == 0) {
    s_actn = 0;
    s_pruned = 0;
    s_wedges = 0;
  }
  Ctrl *ctrl = a.ctrl;
  if (tid0 == 0) {
    s_exit = ld_rlx(&ctrl->status) != 0;
    s_solve = -1;
    s_idle = 0;
    s_gmin = 0;
  }
  __syncthreads();
  if (s_exit) return;

  const unsigned long long t_start = wall_clock64();
  const unsigned long long window = a.ctrl->window;  // fixed before the launch
  int rounds = 0;
  // counters of this workgroup (thread 0), added to the stats once at exit
  unsigned long long st_tot = 0, st_upd = 0, st_cross = 0, st_exp = 0, st_batches = 0;
  int stay = -1;  // unit kept from the previous batch (still holding work)
  uint32_t mixkey = blockIdx.x * 0x85EBCA6Bu;
  unsigned long long umv[4], um0[4];

  for (;;) {
    // thread-derived offsets are recomputed every batch rather than held live
    const int tid = opaque_v(tid0);
    const int lane = tid & (WAVE - 1);
    const int wid = tid / WAVE;
    // ------------------------------------------------------------- 1. pick
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
    mixkey += 0x27D4EB2Fu;
    uint32_t *const abits = opaque(a.abits);
    unsigned long long *const unit_min = opaque(a.unit_min);
    if (stay < 0) {
      // global least pending minimum over the active units (an active unit
      // whose minimum is not known yet counts as +inf and stays eligible)
      unsigned long long gl = ~0ull;
      uint32_t act0 = 0;
      for (int u0 = 0; u0 < a.nunits; u0 += BS * 4) {
        uint32_t wv[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int u = u0 + j * BS + tid;
          wv[j] = u < a.nunits ? ld_rlx(&abits[abw(u)]) : 0u;
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int u = u0 + j * BS + tid;
          umv[j] = ~0ull;
          const bool act = u < a.nunits && (wv[j] & abit(u)) != 0u;
          if (act) umv[j] = ld_rlx(&unit_min[u]);
          if (u0 == 0) {
            um0[j] = umv[j];
            act0 |= (uint32_t)act << j;
          }
        }
#pragma unroll
        for (int j = 0; j < 4; j++) gl = umv[j] < gl ? umv[j] : gl;
      }
      gl = wave_min(gl);
      if (lane == 0) s_red[wid] = gl;
      __syncthreads();
      unsigned long long gmin = s_red[0];
#pragma unroll
      for (int k = 1; k < NW; k++) gmin = s_red[k] < gmin ? s_red[k] : gmin;
      __syncthreads();
      // random choice among the active units within the lag window of gmin
      unsigned long long best = ~0ull;
      for (int u0 = 0; u0 < a.nunits; u0 += BS * 4) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int u = u0 + j * BS + tid;
          bool act;
          unsigned long long d;
          if (u0 == 0) {
            act = (act0 >> j) & 1u;
            d = um0[j];
          } else {
            act = u < a.nunits && (ld_rlx(&abits[abw(u)]) & abit(u)) != 0u;
            d = act ? ld_rlx(&unit_min[u]) : ~0ull;
          }
          if (act && (d == ~0ull || gmin == ~0ull || window == DELTA_INF ||
                      Dist<WT>::within(d, gmin, window))) {
            const unsigned long long key = unit_mix((uint32_t)u, mixkey);
            best = key < best ? key : best;
          }
        }
      }
      best = wave_min(best);
      if (lane == 0) s_red[wid] = best;
      __syncthreads();
      if (tid == 0) {
        // try the per-wave picks in increasing key order (unrolled selection)
        uint32_t tried = 0;
        for (int it = 0; it < NW; it++) {
          unsigned long long bk = ~0ull;
          int bi = -1;
#pragma unroll
          for (int k = 0; k < NW; k++) {
            const unsigned long long ck = s_red[k];
            if (!((tried >> k) & 1u) && ck < bk) {
              bk = ck;
              bi = k;
            }
          }
          if (bi < 0) break;
          tried |= 1u << bi;
          const int u = (int)unit_unmix((uint32_t)bk, mixkey);
          const uint32_t mb = abit(u);
          if (aand_acq(&abits[abw(u)], ~mb) & mb) {
            s_unit = u;
            s_gmin = gmin;
            break;
          }
        }
      }
      __syncthreads();
    } else if (tid == 0) {
      s_unit = stay;
    }
    if (stay < 0 && s_unit < 0 && tid == 0) s_idle = s_idle < 7 ? s_idle + 1 : 7;
    if (s_unit >= 0 && tid == 0) s_idle = 0;
    __syncthreads();
    const int unit = uni(s_unit);
    if (unit < 0) {
      // idle: finished when no work is pending anywhere
      if (tid == 0 && ld_rlx(&ctrl->work) <= 0) {
        st_rlx(&ctrl->done, 1u);
        s_exit = 1;
      }
      __syncthreads();
      if (s_exit) break;
      if constexpr (IPRUNE) {
        // no unit to settle: prune a chunk of vertices instead, if any is left
        if (tid == 0) {
          s_ptask = ld_rlx(&ctrl->prune_next) < a.prune_tasks ? aadd(&ctrl->prune_next, 1)
                                                               : a.prune_tasks;
          if (s_ptask < a.prune_tasks && s_solve != 0) {
            s_solve = 0;
            s_desc = a.desc[0];
          }
        }
        __syncthreads();
        const int task = uni(s_ptask);
        if (task < a.prune_tasks) {
          const int n = uni(s_desc.n);
          const int m = uni(s_desc.m);
          const int bsize = uni(s_desc.bsize);
          const int32_t *__restrict__ row_ptr = uni_ptr(s_desc.row_ptr);
          const int32_t *__restrict__ col = uni_ptr(s_desc.col);
          const uint32_t *__restrict__ wgt = uni_ptr(s_desc.w);
          const int u0 = task * PRUNE_CHUNK;
          const int u1 = min(n, u0 + PRUNE_CHUNK);
          for (int u = u0; u < u1; u++) {
            const int r0 = row_ptr[u], r1 = row_ptr[u + 1];
            const int deg = r1 - r0;
            if (r0 < 0 || r1 > m || deg < 2 || deg > PT_SLOTS / 2) continue;  // uniform
            const int pu = u / bsize;
            for (int i = tid; i < PT_SLOTS; i += BS) {
              s_pk[i] = -1;
              s_pc[i] = ~0ull;
            }
            if (tid == 0) s_pm = 0;
            __syncthreads();
            // heads of u into the table; middles in u's partition staged
            for (int i = tid; i < deg; i += BS) {
              const int x = col[r0 + i];
              if ((unsigned)x >= (unsigned)n) continue;
              pt_insert(s_pk, x);
              if (x != u && x / bsize == pu) {
                const int y0 = row_ptr[x], y1 = row_ptr[x + 1];
                const int k = atomicAdd(&s_pm, 1);
                s_v[k] = x;
                s_rs[k] = y0;
                s_off[k] = (y0 < 0 || y1 < y0 || y1 > m) ? 0 : y1 - y0;
                s_d[k] = wgt[r0 + i];
              }
            }
            __syncthreads();
            const int nm = uni(s_pm);  // <= deg <= FCAP
            int degs[EPT];
            int lsum = 0;
#pragma unroll
            for (int j = 0; j < EPT; j++) {
              const int k = tid * EPT + j;
              degs[j] = k < nm ? s_off[k] : 0;
              lsum += degs[j];
            }
            int tot;
            int run = block_excl_scan1<BS>(lsum, s_ws, &tot);
#pragma unroll
            for (int j = 0; j < EPT; j++) {
              const int k = tid * EPT + j;
              if (k < nm) s_off[k] = run;
              run += degs[j];
            }
            __syncthreads();
            tot = uni(tot);
            if (tot == 0 || tot > PRUNE_MAX_WEDGES) continue;  // uniform
            // every two-arc path u -> y -> x2: min-combine its cost into x2
            for (int idx = tid; idx < tot; idx += BS) {
              int lo = 0, hi = nm - 1;  // last k with s_off[k] <= idx
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= idx) lo = mid;
                else hi = mid - 1;
              }
              const int e2 = s_rs[lo] + (idx - s_off[lo]);
              const int x2 = col[e2];
              if (x2 == s_v[lo]) continue;  // the middle must differ from the head
              const int slot = pt_find(s_pk, x2);
              if (slot >= 0) atomicMin(&s_pc[slot], pair_cost<WT>(s_d[lo], wgt[e2]));
            }
            __syncthreads();
            // each arc of u against its head's least detour
            unsigned long long np = 0;
            for (int i = tid; i < deg; i += BS) {
              const int e = r0 + i;
              const int x = col[e];
              if ((unsigned)x >= (unsigned)n) continue;
              const int slot = pt_find(s_pk, x);
              if (slot >= 0 && pair_beats<WT>(s_pc[slot], wgt[e])) {
                __hip_atomic_fetch_and(&a.keepbits[e >> 5], ~(1u << (e & 31)), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                np++;
              }
            }
            np = wave_sum(np);
            if (lane == 0 && np) atomicAdd(&s_pruned, np);
            if (tid == 0) s_wedges += tot;
            __syncthreads();
          }
          if (tid == 0) s_idle = 0;
          continue;
        }
      }
      for (int k = 0; k < (1 << s_idle); k++) __builtin_amdgcn_s_sleep(16);
      continue;
    }

    if (tid == 0) {
      const int sv = a.unit_solve[unit];
      if (sv != s_solve) {
        s_solve = sv;
        s_desc = a.desc[sv];
      }
      // pushes from now on lower this with atomic min; the gather below
      // covers every inbox bit set before this store
      st_rlx(&unit_min[unit], LABEL_INF);
      s_nlist = 0;
      s_cnt = 0;
      s_far = ~0ull;
      s_lmin = ~0ull;
      s_upd = 0;
      s_cross = 0;
      s_new = 0;
      s_tot = 0;
      s_exp = 0;
    }
    __syncthreads();
    const int n = uni(s_desc.n);
    const int m = uni(s_desc.m);
    const int bsize = uni(s_desc.bsize);
    const int source = uni(s_desc.source);
    const int unit0 = uni(s_desc.unit0);
    const unsigned long long delta = uni64(s_desc.delta);
    const int32_t *__restrict__ row_ptr = uni_ptr(s_desc.row_ptr);
    const int32_t *__restrict__ col = uni_ptr(s_desc.col);
    const uint32_t *__restrict__ wgt = uni_ptr(s_desc.w);
    unsigned long long *label = uni_ptr(s_desc.label);
    uint32_t *dirty = uni_ptr(s_desc.dirty);
    const int part = unit - unit0;
    const int vlo = part * bsize;
    const int vhi = min(n, vlo + bsize);
    const int wlo = vlo >> 5;
    const int whi = (vhi - 1) >> 5;

    // ------------------------------------------------ 2. gather the inbox
    // Claim every inbox bit of the unit (one atomic and-not per word, whose
    // result lists the claimed vertices), then load their labels: a label
    // lowered after the claim sets its bit again.  Vertices beyond FCAP or
    // outside the lowest bucket go back to the inbox.
    long long claimed = 0;  // thread 0: inbox bits taken by this batch
    for (int wb = wlo; wb <= whi; wb += BS) {
      const int wi = wb + tid;
      uint32_t bits = 0;
      if (wi <= whi) {
        uint32_t mask = ~0u;
        if (wi == wlo) mask &= ~0u << (vlo & 31);
        if (wi == whi) {
          const int hb = (vhi - 1) & 31;
          mask &= hb == 31 ? ~0u : ((1u << (hb + 1)) - 1u);
        }
        if (ld_rlx(&dirty[wi]) & mask) bits = aand_acq(&dirty[wi], ~mask) & mask;
      }
      int tot;
      const int before = s_nlist;
      // one barrier: s_ws is next written after this iteration's last barrier
      int j = before + block_excl_scan1<BS>(__popc(bits), s_ws, &tot);
      uint32_t back = 0;
      for (uint32_t b = bits; b; b &= b - 1) {
        if (j < FCAP) s_rs[j] = wi * 32 + __ffs(b) - 1;
        else back |= b & (~b + 1u);
        j++;
      }
      if (back) {
        const uint32_t ob = aor(&dirty[wi], back);
        atomicAdd(&s_new, (unsigned int)__popc(back & ~ob));
      }
      if (tid == 0) {
        s_nlist = before + tot;
        claimed += tot;
      }
      __syncthreads();
      if (s_nlist >= FCAP) break;
    }
    const int nlist = uni(min(s_nlist, FCAP));
    const bool trunc = s_nlist > FCAP || (s_nlist == FCAP);
    if (nlist == 0) {
      // nothing pending in the unit any more (taken by another workgroup)
      stay = -1;
      __syncthreads();
      continue;
    }
    unsigned long long lmin = ~0ull;
    for (int k0 = 0; k0 < nlist; k0 += BS * 4) {
      unsigned long long lab[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int k = k0 + j * BS + tid;
        lab[j] = k < nlist ? ld_rlx(&label[s_rs[k]]) : ~0ull;
      }
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int k = k0 + j * BS + tid;
        if (k < nlist) {
          const uint32_t dv = (uint32_t)(lab[j] >> 32);
          s_d[k] = dv;
          lmin = dv < lmin ? dv : lmin;
        }
      }
    }
    for (int i = tid; i <= whi - wlo; i += BS) s_fm[i] = 0u;
    lmin = wave_min(lmin);
    if (lane == 0) s_red[wid] = lmin;
    __syncthreads();
    unsigned long long umin = s_red[0];
#pragma unroll
    for (int k = 1; k < NW; k++) umin = s_red[k] < umin ? s_red[k] : umin;
    unsigned long long T = 0;  // end of the bucket being settled (bucket modes)
    int cnt = 0;               // its claimed vertices
    if constexpr (!HEAP) {
      T = Dist<WT>::bucket_end(umin, delta);
      // the lowest bucket is the frontier (with the distances just loaded);
      // the rest goes back to the inbox, one atomic or per word
      unsigned long long far = ~0ull;
      for (int k = tid; k < nlist; k += BS) {
        const uint32_t dv = s_d[k];
        const int v = s_rs[k];
        if ((unsigned long long)dv < T) {
          const int slot = atomicAdd(&s_cnt, 1);
          s_v[slot] = v;
          s_vd[slot] = dv;
        } else {
          far = dv < far ? dv : far;
          atomicOr(&s_fm[(v >> 5) - wlo], 1u << (v & 31));
        }
      }
      far = wave_min(far);
      if (lane == 0 && far != ~0ull) atomicMin(&s_far, far);
      __syncthreads();
      unsigned int putback = 0;
      for (int i = tid; i <= whi - wlo; i += BS) {
        const uint32_t fb = s_fm[i];
        if (fb) putback += __popc(fb & ~aor(&dirty[wlo + i], fb));
      }
      putback = wave_sum(putback);
      if (lane == 0 && putback) atomicAdd(&s_new, putback);
      cnt = uni(s_cnt);
    }

    // ---------------------------------------- 3-4. settle the bucket locally
    // Rounds: stage the frontier's rows, relax every arc; heads in this
    // partition that land in the current bucket form the next round's
    // frontier in LDS (deduplicated by an LDS bitmap) instead of going
    // through the inbox, so the partition settles its bucket in one batch.
    // The batch first raises the pending count by RAISE, more than the inbox
    // bits all its rounds can set (at most m per round, MAX_ROUNDS_PER_BATCH
    // rounds), and returns the surplus once at the end.
    long long raised = 0;  // thread 0 only

    // ------------------------------------------- 3-4. heap batch (SOLVE_HEAP)
    // Alg. 3 taken literally inside the partition: every claimed inbox
    // vertex goes into an LDS binary heap keyed by (distance, vertex); the
    // batch pops the least entry, relaxes its arcs with the whole workgroup,
    // pushes every head of this partition whose distance it lowered, and
    // marks every lowered head of another partition in its owner's inbox
    // (the message).  Lazy deletion: an entry whose vertex's label has
    // dropped below its key since it was pushed is skipped (a lower entry,
    // or an inbox bit, exists for that drop).  The batch drains the heap or
    // stops after MAX_ROUNDS_PER_BATCH pops; entries left go back to the
    // inbox.  Heap or list overflow sends a head to the inbox instead.
    if constexpr (HEAP) {
      if (tid == 0) {
        // raised before any inbox bit of this batch is published (the
        // returned value is consumed so the add completes first)
        const long long before = aadd(&ctrl->work, RAISE);
        raised = RAISE;
        int hn = 0;
        for (int k = 0; k < nlist; k++)
          s_heap[hn++] = ((unsigned long long)s_d[k] << 32) | (uint32_t)s_rs[k];
        for (int i = hn / 2 - 1; i >= 0; i--) heap_down(s_heap, hn, i);
        s_hn = before == LLONG_MIN ? 0 : hn;
      }
      __syncthreads();
      for (int pops = 0; pops < MAX_ROUNDS_PER_BATCH; pops++) {
        if (tid == 0) {
          int u = -1, r0 = 0, r1 = 0;
          uint32_t du = 0;
          int hn = s_hn;
          while (hn > 0) {
            const unsigned long long key = s_heap[0];
            hn--;
            if (hn > 0) {
              s_heap[0] = s_heap[hn];
              heap_down(s_heap, hn, 0);
            }
            const int v = (int)(uint32_t)key;
            const uint32_t dk = (uint32_t)(key >> 32);
            if ((uint32_t)(ld_rlx(&label[v]) >> 32) < dk) continue;  // stale entry
            u = v;
            du = dk;
            break;
          }
          s_hn = hn;
          if (u >= 0) {
            r0 = row_ptr[u];
            r1 = row_ptr[u + 1];
            if (r0 < 0 || r1 < r0 || r1 > m) {
              set_status(&ctrl->status, SSSP_ERR_CSR);
              r0 = 0;
              r1 = 0;
            }
          }
          s_hu = u;
          s_hdu = du;
          s_hr0 = r0;
          s_hr1 = r1;
          s_ncnt = 0;
        }
        __syncthreads();
        const int u = uni(s_hu);
        if (u < 0) break;
        const uint32_t du = (uint32_t)uni((int)s_hdu);
        const int r0 = uni(s_hr0);
        const int deg = uni(s_hr1) - r0;
        unsigned int upd = 0, cross = 0, nnew = 0;
        unsigned long long pmin = ~0ull;
        for (int b0 = 0; b0 < deg; b0 += BS * U) {
          int e[U], v[U];
          uint32_t wv[U], nd[U];
          bool act[U];
#pragma unroll
          for (int j = 0; j < U; j++) {
            const int idx = b0 + j * BS + tid;
            act[j] = idx < deg;
            if (act[j]) e[j] = r0 + idx;
          }
#pragma unroll
          for (int j = 0; j < U; j++)
            if (act[j]) {
              v[j] = col[e[j]];
              wv[j] = wgt[e[j]];
            }
          unsigned long long pk[U], cur[U];
#pragma unroll
          for (int j = 0; j < U; j++) {
            if (!act[j]) continue;
            if ((unsigned)v[j] >= (unsigned)n) {
              set_status(&ctrl->status, SSSP_ERR_CSR);
              act[j] = false;
              continue;
            }
            bool ovf;
            nd[j] = Dist<WT>::add(du, wv[j], ovf);
            if (ovf) {
              st_rlx(&ctrl->ovf, 1u);  // decided after the solve, as in the bucket modes
              act[j] = false;
              continue;
            }
            if (v[j] == source) {
              act[j] = false;
              continue;
            }
            pk[j] = ((unsigned long long)nd[j] << 32) | (uint32_t)e[j];
            cur[j] = ld_rlx(&label[v[j]]);
          }
#pragma unroll
          for (int j = 0; j < U; j++) {
            if (act[j] && pk[j] < cur[j]) cur[j] = amin(&label[v[j]], pk[j]);
            else act[j] = false;
          }
          bool inbox[U];
#pragma unroll
          for (int j = 0; j < U; j++) {
            inbox[j] = false;
            if (!act[j] || (uint32_t)(cur[j] >> 32) <= nd[j]) {
              act[j] = false;
              continue;
            }
            upd++;
            if (v[j] / bsize != part) {
              cross++;
              inbox[j] = true;
            } else {
              // pq.push(v): one entry per lowering, pushed after the row
              const int slot = atomicAdd(&s_ncnt, 1);
              if (slot < FCAP) {
                s_nv[slot] = v[j];
                s_vd[slot] = nd[j];
              } else {
                inbox[j] = true;
              }
            }
          }
          uint32_t ob[U];
#pragma unroll
          for (int j = 0; j < U; j++)
            if (inbox[j]) ob[j] = aor(&dirty[v[j] >> 5], 1u << (v[j] & 31));
#pragma unroll
          for (int j = 0; j < U; j++) {
            if (!inbox[j] || ((ob[j] >> (v[j] & 31)) & 1u)) continue;  // already pending
            nnew++;
            const int q = v[j] / bsize;
            if (q != part) {
              const int gu = unit0 + q;
              if (!act_defer(s_actk, s_actd, &s_actn, gu, nd[j])) {
                amin(&unit_min[gu], (unsigned long long)nd[j]);
                aor(&abits[abw(gu)], abit(gu));
              }
            } else {
              pmin = nd[j] < pmin ? nd[j] : pmin;
            }
          }
        }
        upd = wave_sum(upd);
        cross = wave_sum(cross);
        nnew = wave_sum(nnew);
        pmin = wave_min(pmin);
        if (lane == 0) {
          if (upd) atomicAdd(&s_upd, upd);
          if (cross) atomicAdd(&s_cross, cross);
          if (nnew) atomicAdd(&s_new, nnew);
          if (pmin != ~0ull) atomicMin(&s_lmin, pmin);
        }
        if (tid == 0) {
          s_tot += deg;
          s_exp += 1;
        }
        __syncthreads();
        if (tid == 0) {
          // push the lowered local heads; a full heap sends them to the inbox
          const int k = min(s_ncnt, FCAP);
          int hn = s_hn;
          unsigned int spill = 0;
          unsigned long long smin = ~0ull;
          for (int i = 0; i < k; i++) {
            const unsigned long long key =
                ((unsigned long long)s_vd[i] << 32) | (uint32_t)s_nv[i];
            if (hn < HCAP) {
              heap_up(s_heap, hn, key);
              hn++;
            } else {
              const int v2 = s_nv[i];
              const uint32_t bit = 1u << (v2 & 31);
              if (!(aor(&dirty[v2 >> 5], bit) & bit)) spill++;
              smin = s_vd[i] < smin ? s_vd[i] : smin;
            }
          }
          s_hn = hn;
          if (spill) s_new += spill;
          if (smin != ~0ull) s_lmin = smin < s_lmin ? smin : s_lmin;
        }
        if (s_actn <= ACT_FEW) {  // few units pushed into: wake them now
          for (int i = tid; i < ACT_SLOTS; i += BS) {
            const int gu = s_actk[i];
            if (gu >= 0) {
              amin(&unit_min[gu], (unsigned long long)s_actd[i]);
              aor(&abits[abw(gu)], abit(gu));
              s_actk[i] = -1;
              s_actd[i] = 0xFFFFFFFFu;
            }
          }
          __syncthreads();
          if (tid == 0) s_actn = 0;
        }
        __syncthreads();
      }
      // entries left in the heap go back to the inbox (stale ones need not)
      unsigned int back = 0;
      unsigned long long bmin = ~0ull;
      const int hleft = uni(s_hn);
      for (int i = tid; i < hleft; i += BS) {
        const unsigned long long key = s_heap[i];
        const int v2 = (int)(uint32_t)key;
        const uint32_t dk = (uint32_t)(key >> 32);
        if ((uint32_t)(ld_rlx(&label[v2]) >> 32) < dk) continue;
        const uint32_t bit = 1u << (v2 & 31);
        if (!(aor(&dirty[v2 >> 5], bit) & bit)) back++;
        bmin = dk < bmin ? dk : bmin;
      }
      back = wave_sum(back);
      bmin = wave_min(bmin);
      if (lane == 0) {
        if (back) atomicAdd(&s_new, back);
        if (bmin != ~0ull) atomicMin(&s_lmin, bmin);
      }
      __syncthreads();
    } else {
      int cur_cnt = cnt;
      int nround = 0;
      for (;;) {
        if (tid == 0) {
          if (nround == 0) {
            // the returned value is consumed so that the add has completed
            // before thread 0 reaches the barrier below (no inbox bit of this
            // batch is published before that barrier)
            const long long before = aadd(&ctrl->work, RAISE);
            raised = RAISE;
            s_ncnt = before == LLONG_MIN ? 1 : 0;
          } else {
            s_ncnt = 0;
          }
        }
        for (int k0 = 0; k0 < cur_cnt; k0 += BS * 4) {
          unsigned long long lab[4];
          int rs[4], re[4];
#pragma unroll
          for (int j = 0; j < 4; j++) {
            const int k = k0 + j * BS + tid;
            if (k < cur_cnt) {
              const int u = s_v[k];
              // round 0: the labels loaded after the claim; later rounds: the
              // current label of each LDS-queued vertex
              lab[j] = nround == 0 ? (unsigned long long)s_vd[k] << 32 : ld_rlx(&label[u]);
              rs[j] = row_ptr[u];
              re[j] = row_ptr[u + 1];
            }
          }
#pragma unroll
          for (int j = 0; j < 4; j++) {
            const int k = k0 + j * BS + tid;
            if (k < cur_cnt) {
              int r0 = rs[j], r1 = re[j];
              if (r0 < 0 || r1 < r0 || r1 > m) {
                set_status(&ctrl->status, SSSP_ERR_CSR);
                r0 = 0;
                r1 = 0;
              }
              s_d[k] = (uint32_t)(lab[j] >> 32);
              s_rs[k] = r0;
              s_off[k] = r1 - r0;
            }
          }
        }
        __syncthreads();
        int degs[EPT];
        int lsum = 0;
#pragma unroll
        for (int j = 0; j < EPT; j++) {
          const int k = tid * EPT + j;
          degs[j] = k < cur_cnt ? s_off[k] : 0;
          lsum += degs[j];
        }
        int tot;
        int run = block_excl_scan1<BS>(lsum, s_ws, &tot);  // s_ws reused after later barriers
#pragma unroll
        for (int j = 0; j < EPT; j++) {
          const int k = tid * EPT + j;
          if (k < cur_cnt) s_off[k] = run;
          run += degs[j];
        }
        if (tid == 0) s_off[cur_cnt] = tot;
        __syncthreads();

        unsigned int upd = 0, cross = 0, nnew = 0;
        unsigned long long pmin = ~0ull;
        int hint = 0;
        for (int b0 = 0; b0 < tot; b0 += BS * U) {
          int e[U], v[U];
          uint32_t du[U], wv[U], nd[U];
          bool act[U];
#pragma unroll
          for (int j = 0; j < U; j++) {
            const int idx = b0 + j * BS + tid;
            act[j] = idx < tot;
            if (act[j]) {
              // last k with s_off[k] <= idx, galloping up from the previous k
              int lo = hint, step = 1;
              while (lo + step < cur_cnt && s_off[lo + step] <= idx) {
                lo += step;
                step <<= 1;
              }
              int hi = min(lo + step, cur_cnt) - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= idx) lo = mid;
                else hi = mid - 1;
              }
              hint = lo;
              e[j] = s_rs[lo] + (idx - s_off[lo]);
              du[j] = s_d[lo];
            }
          }
          uint32_t kb[U];
#pragma unroll
          for (int j = 0; j < U; j++)
            if (act[j]) {
              v[j] = col[e[j]];
              wv[j] = wgt[e[j]];
              // arcs deleted by idle-time pruning are not relaxed (a plain
              // load: a stale bit only relaxes a deleted arc, which is harmless)
              if constexpr (IPRUNE) kb[j] = a.keepbits[e[j] >> 5];
            }
          unsigned long long pk[U], cur[U];
#pragma unroll
          for (int j = 0; j < U; j++) {
            if (!act[j]) continue;
            if constexpr (IPRUNE) {
              if (!((kb[j] >> (e[j] & 31)) & 1u)) {
                act[j] = false;
                continue;
              }
            }
            if ((unsigned)v[j] >= (unsigned)n) {
              set_status(&ctrl->status, SSSP_ERR_CSR);
              act[j] = false;
              continue;
            }
            bool ovf;
            nd[j] = Dist<WT>::add(du[j], wv[j], ovf);
            if (ovf) {
              // a candidate that does not fit is no shorter path to anything
              // that fits: skip it.  Whether a final distance overflowed is
              // decided after the fixed point (in k_epilogue); this flag only
              // says that the check has to look.
              st_rlx(&ctrl->ovf, 1u);
              act[j] = false;
              continue;
            }
            if (v[j] == source) {
              act[j] = false;
              continue;
            }
            pk[j] = ((unsigned long long)nd[j] << 32) | (uint32_t)e[j];
            cur[j] = ld_rlx(&label[v[j]]);
          }
          if constexpr (XBUF) {
            // cross-partition candidates that beat the current label wait in
            // the LDS buffer (applied once per distinct head at the flush)
#pragma unroll
            for (int j = 0; j < U; j++)
              if (act[j] && pk[j] < cur[j] && v[j] / bsize != part &&
                  xb_insert(s_xbk, s_xbv, &s_xbn, v[j], pk[j]))
                act[j] = false;
          }
#pragma unroll
          for (int j = 0; j < U; j++) {
            if (act[j] && pk[j] < cur[j]) cur[j] = amin(&label[v[j]], pk[j]);
            else act[j] = false;
          }
          // lowered distances: same partition and same bucket -> next round in
          // LDS; otherwise -> the owner's inbox bit
          bool inbox[U];
#pragma unroll
          for (int j = 0; j < U; j++) {
            inbox[j] = false;
            if (!act[j] || (uint32_t)(cur[j] >> 32) <= nd[j]) {
              act[j] = false;
              continue;
            }
            upd++;
            const int q = v[j] / bsize;
            if (q != part) {
              cross++;
              inbox[j] = true;
            } else if ((unsigned long long)nd[j] < T) {
              const int lv = v[j] - vlo;
              const uint32_t mb = 1u << (lv & 31);
              if (!(atomicOr(&s_mark[lv >> 5], mb) & mb)) {
                const int slot = atomicAdd(&s_ncnt, 1);
                if (slot < FCAP) s_nv[slot] = v[j];
                else {
                  atomicAnd(&s_mark[lv >> 5], ~mb);
                  inbox[j] = true;
                }
              }
            } else {
              inbox[j] = true;
            }
          }
          uint32_t ob[U];
#pragma unroll
          for (int j = 0; j < U; j++)
            if (inbox[j]) ob[j] = aor(&dirty[v[j] >> 5], 1u << (v[j] & 31));
#pragma unroll
          for (int j = 0; j < U; j++) {
            if (!inbox[j] || ((ob[j] >> (v[j] & 31)) & 1u)) continue;  // already pending
            nnew++;
            const int q = v[j] / bsize;
            if (q != part) {
              const int gu = unit0 + q;
              if (!act_defer(s_actk, s_actd, &s_actn, gu, nd[j])) {
                amin(&unit_min[gu], (unsigned long long)nd[j]);
                aor(&abits[abw(gu)], abit(gu));
              }
            } else {
              pmin = nd[j] < pmin ? nd[j] : pmin;
            }
          }
        }
        upd = wave_sum(upd);
        cross = wave_sum(cross);
        nnew = wave_sum(nnew);
        pmin = wave_min(pmin);
        if (lane == 0) {
          if (upd) atomicAdd(&s_upd, upd);
          if (cross) atomicAdd(&s_cross, cross);
          if (nnew) atomicAdd(&s_new, nnew);
          if (pmin != ~0ull) atomicMin(&s_lmin, pmin);
        }
        if (tid == 0) {
          s_tot += tot;
          s_exp += cur_cnt;
        }
        __syncthreads();
        if constexpr (XBUF) {
          if (s_xbn >= SSSP_XB_FLUSH) {  // push out on count
            unsigned int fu = 0, fc = 0, fn = 0;
            xb_flush<BS>(s_xbk, s_xbv, label, dirty, bsize, unit0, unit_min, abits, s_actk, s_actd,
                         &s_actn, fu, fc, fn);
            fu = wave_sum(fu);
            fc = wave_sum(fc);
            fn = wave_sum(fn);
            if (lane == 0) {
              if (fu) atomicAdd(&s_upd, fu);
              if (fc) atomicAdd(&s_cross, fc);
              if (fn) atomicAdd(&s_new, fn);
            }
            __syncthreads();
            if (tid == 0) s_xbn = 0;
          }
        }
        if (s_actn <= ACT_FEW) {  // few units pushed into: wake them now
          for (int i = tid; i < ACT_SLOTS; i += BS) {
            const int gu = s_actk[i];
            if (gu >= 0) {
              amin(&unit_min[gu], (unsigned long long)s_actd[i]);
              aor(&abits[abw(gu)], abit(gu));
              s_actk[i] = -1;
              s_actd[i] = 0xFFFFFFFFu;
            }
          }
          __syncthreads();
          if (tid == 0) s_actn = 0;
        }
        const int ncnt = uni(min(s_ncnt, FCAP));
        nround++;
        if (ncnt == 0) break;
        if (nround >= MAX_ROUNDS_PER_BATCH) {
          // hand the queued vertices back to the inbox (covered by this
          // round's raise) and stop
          unsigned int fl = 0;
          for (int k = tid; k < ncnt; k += BS) {
            const int v2 = s_nv[k];
            const int lv = v2 - vlo;
            atomicAnd(&s_mark[lv >> 5], ~(1u << (lv & 31)));
            const uint32_t bit = 1u << (v2 & 31);
            if (!(aor(&dirty[v2 >> 5], bit) & bit)) fl++;
          }
          fl = wave_sum(fl);
          if (lane == 0 && fl) atomicAdd(&s_new, fl);
          if (tid == 0) atomicMin(&s_lmin, umin);
          __syncthreads();
          break;
        }
        for (int k = tid; k < ncnt; k += BS) {
          const int v2 = s_nv[k];
          const int lv = v2 - vlo;
          atomicAnd(&s_mark[lv >> 5], ~(1u << (lv & 31)));
          s_v[k] = v2;
        }
        cur_cnt = ncnt;
        __syncthreads();
      }
    }

    if constexpr (XBUF) {
      // push out what the batch still buffers (it records wakeups, which
      // are published next)
      if (s_xbn > 0) {
        unsigned int fu = 0, fc = 0, fn = 0;
        xb_flush<BS>(s_xbk, s_xbv, label, dirty, bsize, unit0, unit_min, abits, s_actk, s_actd,
                     &s_actn, fu, fc, fn);
        fu = wave_sum(fu);
        fc = wave_sum(fc);
        fn = wave_sum(fn);
        if (lane == 0) {
          if (fu) atomicAdd(&s_upd, fu);
          if (fc) atomicAdd(&s_cross, fc);
          if (fn) atomicAdd(&s_new, fn);
        }
        __syncthreads();
        if (tid == 0) s_xbn = 0;
      }
    }
    // deferred activations of the units this batch pushed into: published
    // before the settle below returns the batch's surplus of pending work
    for (int i = tid; i < ACT_SLOTS; i += BS) {
      const int gu = s_actk[i];
      if (gu >= 0) {
        amin(&unit_min[gu], (unsigned long long)s_actd[i]);
        aor(&abits[abw(gu)], abit(gu));
        s_actk[i] = -1;
        s_actd[i] = 0xFFFFFFFFu;
      }
    }
    if (tid == 0) s_actn = 0;
    __syncthreads();
    // ------------------------------------------------------ 5. settle
    if (tid == 0) {
      // every consequence of this batch is published: return the surplus
      aadd(&ctrl->work, (long long)s_new - raised - claimed);
      unsigned long long rem = s_far < s_lmin ? s_far : s_lmin;
      if (trunc) rem = umin < rem ? umin : rem;
      s_stay = -1;
      if (rem != ~0ull) {
        amin(&unit_min[unit], rem);
        // keep the unit while its remaining work is within the lag window of
        // the least pending distance seen at the pick; otherwise (or when it
        // overflowed the frontier) let any workgroup take it
        if (!trunc && (window == DELTA_INF || Dist<WT>::within(rem, s_gmin, window)))
          s_stay = unit;
        else
          aor(&abits[abw(unit)], abit(unit));
      }
      st_tot += (unsigned long long)s_tot;
      st_upd += s_upd;
      st_cross += s_cross;
      st_exp += (unsigned long long)s_exp;
      st_batches++;
      if (a.max_rounds > 0 && ++rounds >= a.max_rounds) {
        set_status(&ctrl->status, SSSP_ERR_TIMEOUT);
        st_rlx(&ctrl->done, 1u);
      }
    }
    __syncthreads();
    stay = s_stay;
  }
  if constexpr (IPRUNE) {
    if (threadIdx.x == 0 && a.stats && s_wedges) {
      stat_add(&a.stats->edges_pruned, s_pruned);
      stat_add(&a.stats->wedges, s_wedges);
    }
  }
  if (threadIdx.x == 0 && a.stats && st_batches) {
    stat_add(&a.stats->edges_relaxed, st_tot);
    stat_add(&a.stats->label_updates, st_upd);
    stat_add(&a.stats->cross_updates, st_cross);
    stat_add(&a.stats->vertices_expanded, st_exp);
    stat_add(&a.stats->batches, st_batches);
  }
}

// --------------------------------------------------------------- epilogue
// Unpacks labels: dist = high word (sentinel kept), pred_edge = low word
// (-1 for none), pred = tail of pred_edge by binary search in row_ptr.
//
// It also decides overflow, but only when the solve met a relaxation
// candidate that did not fit the distance type (Ctrl::ovf).  The solve
// skipped those candidates, so its fixed point is the true distance wherever
// that fits and +inf where the true distance is finite but too large.  Some
// true distance is too large exactly when an arc leads from a reached vertex
// to a vertex left at +inf (on a shortest path to such a vertex, the first
// vertex whose distance does not fit has a reached predecessor): each thread
// scans the rows of its reached vertices for such an arc.  Not after another
// error, since the labels and the CSR may then be unusable.
template <int WT>
__global__ void k_epilogue(SolveArgs a) {
  const int s = blockIdx.y;
  const SolveDesc d = a.desc[s];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  const bool check = ld_rlx(&a.ctrl->ovf) != 0u && ld_rlx(&a.ctrl->status) == 0;
  bool over = false;
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
      if (check && !over) {
        const int r0 = d.row_ptr[v], r1 = d.row_ptr[v + 1];
        if (r0 >= 0 && r1 >= r0 && r1 <= d.m)
          for (int e = r0; e < r1 && !over; e++) {
            const int x = d.col[e];
            over = (unsigned)x < (unsigned)d.n && d.label[x] == LABEL_INF;
          }
      }
    }
    dist[v] = dv;
    if (d.pred) d.pred[v] = pv;
    if (d.pred_edge) d.pred_edge[v] = pe;
  }
  if (over) {
    set_status(&a.ctrl->status, SSSP_ERR_OVERFLOW);
    if (a.stats) set_status(&a.stats->status, SSSP_ERR_OVERFLOW);
  }
  if (s == 0 && t == 0 && a.stats) {
    // the stats were cleared before the solve; a block that finds an
    // overflow sets both words, so copy only a status that is already set
    set_status(&a.stats->status, ld_rlx(&a.ctrl->status));
    a.stats->num_partitions = d.nparts;
    a.stats->delta_bits = d.delta;
  }
}

// ------------------------------------------------------------- validation
// CSR and weight checks; the first violation is written to *status.  Rows
// are checked for sortedness one wave per row (rows can be very long).
__global__ void k_validate(const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                           int n, int m, int wtype, int need_sorted, int need_positive,
                           int32_t *status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  if (t == 0 && (row_ptr[0] != 0 || row_ptr[n] != m)) set_status(status, SSSP_ERR_CSR);
  for (int u = t; u < n; u += stride) {
    const int a = row_ptr[u], b = row_ptr[u + 1];
    if (a > b || a < 0 || b > m) set_status(status, SSSP_ERR_CSR);
  }
  if (need_sorted) {
    const int wave = t / WAVE;
    const int nwaves = stride / WAVE;
    for (int u = wave; u < n; u += nwaves) {
      const int a = row_ptr[u], b = row_ptr[u + 1];
      if (a > b || a < 0 || b > m) continue;
      bool bad = false;
      for (int e = a + 1 + lane_id(); e < b; e += WAVE) bad |= col[e] < col[e - 1];
      if (__ballot(bad) && lane_id() == 0) set_status(status, SSSP_ERR_UNSORTED);
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

hipError_t launch_auto_delta(const SolveArgs &a, int wtype, int nsolves, hipStream_t st) {
  if (wtype == SSSP_W_U32)
    hipLaunchKernelGGL(k_auto_delta<SSSP_W_U32>, dim3(nsolves), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_auto_delta<SSSP_W_F32>, dim3(nsolves), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_init(const SolveArgs &a, int nsolves, int max_n, hipStream_t st) {
  const int kwords = a.keepbits ? (a.desc_m0 + 31) / 32 : 0;
  int gb = ((kwords > a.nabw ? kwords : a.nabw) + 255) / 256;
  gb = gb < 1 ? 1 : (gb > 256 ? 256 : gb);
  hipLaunchKernelGGL(k_init_global, dim3(gb), dim3(256), 0, st, a, nsolves);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int bx = (max_n + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 1024 ? 1024 : bx);
  hipLaunchKernelGGL(k_init, dim3(bx, nsolves), dim3(256), 0, st, a);
  return hipGetLastError();
}

// The kernel instance for (weight type, block size, mode): launched, or
// asked for its residency.
template <int WT, int BS, int MODE>
static hipError_t solve_kernel_op(const SolveArgs *a, int grid, hipStream_t st, int *per_cu) {
  if (per_cu) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_solve<WT, BS, MODE>,
                                                                  BS, 0);
  hipLaunchKernelGGL((k_solve<WT, BS, MODE>), dim3(grid), dim3(BS), 0, st, *a);
  return hipGetLastError();
}

template <int WT, int BS>
static hipError_t solve_kernel_mode(int mode, const SolveArgs *a, int grid, hipStream_t st,
                                    int *per_cu) {
  if (mode == SOLVE_BUFFERED) return solve_kernel_op<WT, BS, SOLVE_BUFFERED>(a, grid, st, per_cu);
  if (mode == SOLVE_HEAP) return solve_kernel_op<WT, BS, SOLVE_HEAP>(a, grid, st, per_cu);
  if (mode == SOLVE_IDLE_PRUNE)
    return solve_kernel_op<WT, BS, SOLVE_IDLE_PRUNE>(a, grid, st, per_cu);
  return solve_kernel_op<WT, BS, SOLVE_BUCKETS>(a, grid, st, per_cu);
}

template <int WT>
static hipError_t solve_kernel_bs(int bs, int mode, const SolveArgs *a, int grid, hipStream_t st,
                                  int *per_cu) {
  if (bs == 256) return solve_kernel_mode<WT, 256>(mode, a, grid, st, per_cu);
  if (bs == 512) return solve_kernel_mode<WT, 512>(mode, a, grid, st, per_cu);
  return solve_kernel_mode<WT, 1024>(mode, a, grid, st, per_cu);
}

hipError_t launch_solve(const SolveArgs &a, int wtype, int bs, int mode, int grid,
                        hipStream_t st) {
  if (wtype == SSSP_W_U32) return solve_kernel_bs<SSSP_W_U32>(bs, mode, &a, grid, st, nullptr);
  return solve_kernel_bs<SSSP_W_F32>(bs, mode, &a, grid, st, nullptr);
}

int solve_max_blocks_per_cu(int wtype, int bs, int mode) {
  int nb = 0;
  const hipError_t e =
      wtype == SSSP_W_U32 ? solve_kernel_bs<SSSP_W_U32>(bs, mode, nullptr, 0, nullptr, &nb)
                          : solve_kernel_bs<SSSP_W_F32>(bs, mode, nullptr, 0, nullptr, &nb);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_keep_out(const SolveArgs &a, hipStream_t st) {
  int blocks = (a.desc_m0 + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
  hipLaunchKernelGGL(k_keep_out, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
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
