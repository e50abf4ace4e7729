// prune.hip -- Trishla triangle pruning (Sec. III-B, Alg. 1) on gfx950.
//
// Arc e = (u,x,W) is deleted when some middle y, y != u and y != x, has arcs
// (u,y,w1) and (y,x,w2) with w1 + w2 < W, tested against the input graph for
// all arcs at once.  The middles of e are N_out(u) intersected with N_in(x).
//
// Edge-centric form: for every arc the shorter of the two lists is scanned
// and every entry probed in a hash table of the longer one (keyed by the
// middle vertex, holding the cheapest parallel arc).  The work is
// sum_e min(|N_out(u)|, |N_in(x)|) probes instead of the
// sum_y indeg(y) * outdeg(y) wedges of the literal per-vertex loop.
//
//  * arcs with |N_out(u)| <= |N_in(x)| ("x-side") are grouped by x and use
//    the table of N_in(x); the others ("u-side") are grouped by u and use
//    the table of N_out(u);
//  * N_in(x) comes from a CSC (in-lists) built here by a counting sort;
//  * a table owner with a short list and little work is handled by one
//    wavefront with a private LDS table; heavier owners are split into
//    workgroup items of about HV_TARGET probes over an LDS table, or over an
//    L2-resident global table when the list exceeds HV_TCAP entries.
//
// Integer costs are summed in 64 bits; fp32 costs are summed in double,
// which decides w1 + w2 < W exactly for fp32 operands (the sum is exact
// unless one operand is below 2^-29 of the other, and then the comparison
// with an fp32 W cannot flip).
#include "internal.hpp"
#include "launch.hpp"

namespace sssp_impl {

constexpr int TB_BS = 1024;
constexpr int TB_NW = TB_BS / WAVE;
constexpr int LT_DEG = 128;          // light owner: list length
constexpr int LT_SLOTS = 256;        // light owner: wave-private hash slots
constexpr int LT_WORK = 8192;        // light owner: probes
constexpr int HV_TCAP = 8192;        // heavy owner: longest list in an LDS table
constexpr int HV_SLOTS = 16384;
constexpr int HV_Q = 1024;           // heavy: queries staged per round
constexpr int HV_TARGET = 1 << 16;   // heavy: probes per item
constexpr int G_UNIT = 64;           // global table sizes are multiples of this
constexpr uint32_t VAL_INF = 0xFFFFFFFFu;

template <int WT> struct Tri;
template <> struct Tri<SSSP_W_U32> {
  __device__ static __forceinline__ bool lt(uint32_t a, uint32_t b, uint32_t W) {
    return (unsigned long long)a + b < (unsigned long long)W;
  }
};
template <> struct Tri<SSSP_W_F32> {
  __device__ static __forceinline__ bool lt(uint32_t a, uint32_t b, uint32_t W) {
    return (double)__uint_as_float(a) + (double)__uint_as_float(b) <
           (double)__uint_as_float(W);
  }
};

struct TbArgs {
  const int32_t *row_ptr;
  const int32_t *col;
  const uint32_t *w;
  int n, m, local, bsize;
  uint8_t *keep;
  int rep;          // R: replicas of every column counter (spreads hub contention)
  int32_t *src;     // m: tail of every arc
  int32_t *cnt;     // n*R: in-degree replicas
  int32_t *cptr;    // n*R+1: CSC offsets (column x starts at cptr[x*R])
  int32_t *cursor;  // n*R: scatter cursors
  int2 *cyw;        // m: CSC entries (tail, cost)
  int32_t *ceid;    // m: CSC -> CSR edge id
  int2 *ryw;        // m: CSR entries (head, cost), packed copy
  int32_t *work;    // 2n: probes of owner i (i < n: in-table of i; else out-table of i-n)
  int32_t *hflag;   // 2n: owner i is heavy
  int32_t *hpos;    // 2n+1: exclusive scan of hflag
  int32_t *hid;     // heavy owners in order
  int32_t *hitems;  // items of heavy owner j
  int32_t *hoff;    // 2n+1: exclusive scan of hitems
  int32_t *gsz;     // 2n: global table size in units of G_UNIT slots (0 = LDS)
  int32_t *goff;    // 2n+1: exclusive scan of gsz
  int32_t *gkey;    // global tables: keys (-1 = empty)
  uint32_t *gval;   //                cheapest parallel arc
  int32_t *tickets; // [0] heavy items, [1] light owners
  int32_t *status;
  sssp_stats *stats;
};

__device__ __forceinline__ uint32_t tb_hash(int y, int bits) {
  return ((uint32_t)y * 2654435761u) >> (32 - bits);
}

__device__ __forceinline__ void tb_insert(int32_t *keys, uint32_t *vals, int mask, int bits,
                                          int y, uint32_t v) {
  uint32_t h = tb_hash(y, bits);
  for (;;) {
    const int old = atomicCAS(&keys[h], -1, y);
    if (old == -1 || old == y) {
      atomicMin(&vals[h], v);
      return;
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ uint32_t tb_probe(const int32_t *keys, const uint32_t *vals, int mask,
                                             int bits, int y) {
  uint32_t h = tb_hash(y, bits);
  for (;;) {
    const int k = keys[h];
    if (k == y) return vals[h];
    if (k == -1) return VAL_INF;
    h = (h + 1) & mask;
  }
}

// Smallest b >= minbits with 2^b >= 2 * len (load factor at most one half).
__device__ __forceinline__ int tb_bits(int len, int minbits) {
  int b = minbits;
  while ((1 << b) < 2 * len) b++;
  return b;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ setup
__global__ void k_tb_status(TbArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *a.status = 0;
    a.tickets[0] = 0;
    a.tickets[1] = 0;
  }
  if (a.stats && blockIdx.x == 0 && threadIdx.x < (int)(sizeof(sssp_stats) / 4))
    reinterpret_cast<uint32_t *>(a.stats)[threadIdx.x] = 0u;
}

__device__ __forceinline__ int cbeg(const TbArgs &a, int x) { return a.cptr[x * a.rep]; }
__device__ __forceinline__ int clen(const TbArgs &a, int x) {
  return a.cptr[(x + 1) * a.rep] - a.cptr[x * a.rep];
}

__global__ void k_tb_zero(TbArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < a.m; e += stride) a.keep[e] = 1;
  const long long nr = (long long)a.n * a.rep;
  for (long long i = t; i < nr; i += stride) {
    a.cnt[i] = 0;
    a.cursor[i] = 0;
  }
  for (int i = t; i < 2 * a.n; i += stride) {
    a.work[i] = 0;
    a.hitems[i] = 0;
  }
}

// One wave per row: the tail of every arc (coalesced stores only).
__global__ void k_tb_tails(TbArgs a) {
  if (*a.status) return;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nwaves = gridDim.x * blockDim.x / WAVE;
  for (int u = wave; u < a.n; u += nwaves) {
    const int re = a.row_ptr[u + 1];
    for (int e = a.row_ptr[u] + lane_id(); e < re; e += WAVE) a.src[e] = u;
  }
}

__device__ __forceinline__ int rep_of(const TbArgs &a, int e) { return e & (a.rep - 1); }

__global__ void k_tb_indeg(TbArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < a.m; e += stride) {
    const int x = a.col[e];
    if ((unsigned)x < (unsigned)a.n) atomicAdd(&a.cnt[(long long)x * a.rep + rep_of(a, e)], 1);
    else set_status(a.status, SSSP_ERR_CSR);
  }
}

// Thread per arc: scatter into the CSC (each arc into its replica's range)
// and write the packed CSR copy.
__global__ void k_tb_fill(TbArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < a.m; e += stride) {
    const int x = a.col[e];
    const int u = a.src[e];
    const uint32_t wv = a.w[e];
    const long long c = (long long)x * a.rep + rep_of(a, e);
    const int pos = a.cptr[c] + atomicAdd(&a.cursor[c], 1);
    a.cyw[pos] = make_int2(u, (int)wv);
    a.ceid[pos] = e;
    a.ryw[e] = make_int2(x, (int)wv);
  }
}

// Adds val into work[key] for runs of equal keys across the wave: one
// atomic per run (keys are nondecreasing along the lanes).
__device__ __forceinline__ void seg_add(int32_t *work, bool active, int key, int val) {
  const int lane = lane_id();
  const int prev = __shfl_up(key, 1, WAVE);
  const int nextk = __shfl_down(key, 1, WAVE);
  const bool nact = __shfl_down((int)active, 1, WAVE) != 0;
  const bool head = lane == 0 || prev != key;
  const unsigned long long heads = __ballot(head);
  const int incl = wave_incl_scan(active ? val : 0);
  const unsigned long long upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
  const int start = 63 - __clzll(upto);
  const int before = __shfl(incl, start > 0 ? start - 1 : 0, WAVE);
  const bool last = lane == 63 || nextk != key || !nact;
  if (active && last) {
    const int sum = incl - (start > 0 ? before : 0);
    if (sum) atomicAdd(&work[key], sum);
  }
}

// Probes each arc costs, charged to its table owner: the u-side arcs of row
// u add |N_in(x)| to owner n+u (one thread per arc), the x-side arcs of
// column x add |N_out(u)| to owner x (one thread per CSC entry).
__global__ void k_tb_work(TbArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  const int mr = (a.m + WAVE - 1) / WAVE * WAVE;  // whole waves stay in the loop
  for (int e = t; e < mr; e += stride) {
    const bool act = e < a.m;
    int u = -1, val = 0;
    if (act) {
      u = a.src[e];
      const int ou = a.row_ptr[u + 1] - a.row_ptr[u];
      const int ix = clen(a, a.col[e]);
      val = ou > ix ? ix : 0;
    }
    seg_add(a.work + a.n, act, u, val);
  }
  for (int p = t; p < mr; p += stride) {
    const bool act = p < a.m;
    int x = -1, val = 0;
    if (act) {
      const int u = a.cyw[p].x;
      x = a.col[a.ceid[p]];
      const int ou = a.row_ptr[u + 1] - a.row_ptr[u];
      val = ou <= clen(a, x) ? ou : 0;
    }
    seg_add(a.work, act, x, val);
  }
}

__device__ __forceinline__ int owner_len(const TbArgs &a, int i) {
  if (i < a.n) return clen(a, i);
  const int u = i - a.n;
  return a.row_ptr[u + 1] - a.row_ptr[u];
}

__global__ void k_tb_classify(TbArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int i = t; i < 2 * a.n; i += stride) {
    const int wk = a.work[i];
    const int len = owner_len(a, i);
    const bool heavy = wk > 0 && (len > LT_DEG || wk > LT_WORK);
    a.hflag[i] = heavy;
    int g = 0;
    if (heavy && len > HV_TCAP) g = (1 << tb_bits(len, 6)) / G_UNIT;
    a.gsz[i] = g;
  }
}

__global__ void k_tb_heavy_list(TbArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int i = t; i < 2 * a.n; i += stride)
    if (a.hflag[i]) {
      const int j = a.hpos[i];
      const int len = owner_len(a, i);
      int items = (a.work[i] + HV_TARGET - 1) / HV_TARGET;
      items = items < 1 ? 1 : (items > len ? len : items);
      a.hid[j] = i;
      a.hitems[j] = items;
    }
}

// One workgroup per heavy owner with a long list: clear its global table and
// insert the list (owners are taken in turn from the heavy list).
__global__ __launch_bounds__(256) void k_tb_gtab(TbArgs a) {
  if (*a.status) return;
  const int nh = a.hpos[2 * a.n];
  for (int j = blockIdx.x; j < nh; j += gridDim.x) {
    const int i = a.hid[j];
    const int g = a.gsz[i];
    if (!g) continue;
    const long long base = (long long)a.goff[i] * G_UNIT;
    const int slots = g * G_UNIT;
    int32_t *key = a.gkey + base;
    uint32_t *val = a.gval + base;
    for (int s = threadIdx.x; s < slots; s += blockDim.x) {
      key[s] = -1;
      val[s] = VAL_INF;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int bits = tb_bits(slots / 2, 6);
    const bool out_list = i >= a.n;
    const int t = out_list ? i - a.n : i;
    const int lb = out_list ? a.row_ptr[t] : cbeg(a, t);
    const int ll = out_list ? a.row_ptr[t + 1] - lb : clen(a, t);
    for (int p = threadIdx.x; p < ll; p += blockDim.x) {
      const int2 yw = out_list ? a.ryw[lb + p] : a.cyw[lb + p];
      if (yw.x != t) tb_insert(key, val, slots - 1, bits, yw.x, (uint32_t)yw.y);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ main
// Owner i: mode X (i < n: table = N_in(x), queries = x-side arcs into x) or
// mode U (i >= n: table = N_out(u), queries = u-side arcs out of u).
struct Owner {
  int mode;        // 0: X, 1: U
  int t;           // x or u
  int lbeg, llen;  // the owner's list (CSC column or CSR row)
};

__device__ __forceinline__ Owner make_owner(const TbArgs &a, int i) {
  Owner o;
  o.mode = i >= a.n;
  o.t = o.mode ? i - a.n : i;
  if (o.mode) {
    o.lbeg = a.row_ptr[o.t];
    o.llen = a.row_ptr[o.t + 1] - o.lbeg;
  } else {
    o.lbeg = cbeg(a, o.t);
    o.llen = clen(a, o.t);
  }
  return o;
}

// Table entry of list position p (middle vertex y, its cost); -1 = skipped
// (the owner's own self-loop is never a middle).
__device__ __forceinline__ int list_key(const TbArgs &a, const Owner &o, int p, uint32_t &v) {
  const int2 yw = o.mode ? a.ryw[p] : a.cyw[p];
  v = (uint32_t)yw.y;
  return yw.x == o.t ? -1 : yw.x;
}

// Query at list position p: scanned list [beg, beg+len), arc cost W, arc id
// and the arc's other end.  len = 0 when the arc belongs to the other side.
struct Query {
  int beg, len;
  uint32_t W;
  int eid, other;
};

__device__ __forceinline__ Query make_query(const TbArgs &a, const Owner &o, int p) {
  Query q;
  if (o.mode == 0) {  // arc (u -> x = t): scan N_out(u) when |N_out(u)| <= |N_in(x)|
    const int2 uw = a.cyw[p];
    const int u = uw.x;
    const int rs = a.row_ptr[u], ou = a.row_ptr[u + 1] - rs;
    q.beg = rs;
    q.len = ou <= o.llen ? ou : 0;
    q.W = (uint32_t)uw.y;
    q.eid = a.ceid[p];
    q.other = u;
  } else {  // arc (u = t -> x): scan N_in(x) when |N_in(x)| < |N_out(u)|
    const int2 xw = a.ryw[p];
    const int x = xw.x;
    const int cs = cbeg(a, x), ix = clen(a, x);
    q.beg = cs;
    q.len = o.llen <= ix ? 0 : ix;
    q.W = (uint32_t)xw.y;
    q.eid = p;
    q.other = x;
  }
  return q;
}

// Scanned element f of a query: middle y and the cost of its half of the
// detour; false when y may not serve as a witness.
__device__ __forceinline__ bool scan_elem(const TbArgs &a, const Owner &o, int other, int f,
                                          int &y, uint32_t &wa) {
  int u, x;
  const int2 yw = o.mode == 0 ? a.ryw[f] : a.cyw[f];
  y = yw.x;
  wa = (uint32_t)yw.y;
  if (o.mode == 0) {  // element of N_out(u): arc u -> y
    u = other;
    x = o.t;
  } else {  // element of N_in(x): arc y -> x
    u = o.t;
    x = other;
  }
  if (y == u || y == x) return false;
  if (a.local && y / a.bsize != u / a.bsize) return false;
  return true;
}

struct TbHeavy {
  int32_t key[HV_SLOTS];
  uint32_t val[HV_SLOTS];
  int32_t qbeg[HV_Q];
  int32_t qoff[HV_Q + 1];
  uint32_t qW[HV_Q];
  int32_t qeid[HV_Q];
  int32_t qother[HV_Q];
};
struct TbLight {
  int32_t key[TB_NW][LT_SLOTS];
  uint32_t val[TB_NW][LT_SLOTS];
  int32_t qbeg[TB_NW][WAVE];
  int32_t qoff[TB_NW][WAVE + 1];
  uint32_t qW[TB_NW][WAVE];
  int32_t qeid[TB_NW][WAVE];
  int32_t qother[TB_NW][WAVE];
};
union TbShared {
  TbHeavy h;
  TbLight l;
};

template <int WT>
__global__ __launch_bounds__(TB_BS) void k_tb_main(TbArgs a) {
  __shared__ TbShared sh;
  __shared__ int s_ws[TB_NW + 1];
  __shared__ int s_t;
  if (*a.status) return;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid / WAVE;
  const int nh = a.hpos[2 * a.n];
  const int total = a.hoff[nh];
  unsigned long long probes = 0;

  // ---------------------------------------------------------- heavy items
  for (;;) {
    if (tid == 0) s_t = atomicAdd(&a.tickets[0], 1);
    __syncthreads();
    const int it = s_t;
    __syncthreads();
    if (it >= total) break;
    int lo = 0, hi = nh - 1;  // last j with hoff[j] <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.hoff[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const int i = a.hid[lo];
    const int k = it - a.hoff[lo];
    const int ni = a.hitems[lo];
    const Owner o = make_owner(a, i);
    const int32_t *tkey;
    const uint32_t *tval;
    int tbits;
    if (a.gsz[i]) {
      const long long base = (long long)a.goff[i] * G_UNIT;
      tkey = a.gkey + base;
      tval = a.gval + base;
      tbits = tb_bits(a.gsz[i] * G_UNIT / 2, 6);
    } else {
      tbits = tb_bits(o.llen, 6);
      for (int s = tid; s < (1 << tbits); s += TB_BS) {
        sh.h.key[s] = -1;
        sh.h.val[s] = VAL_INF;
      }
      __syncthreads();
      for (int p = tid; p < o.llen; p += TB_BS) {
        uint32_t v;
        const int y = list_key(a, o, o.lbeg + p, v);
        if (y >= 0) tb_insert(sh.h.key, sh.h.val, (1 << tbits) - 1, tbits, y, v);
      }
      __syncthreads();
      tkey = sh.h.key;
      tval = sh.h.val;
    }
    const int tmask = (1 << tbits) - 1;
    // this item's share of the owner's list positions, in rounds of HV_Q
    const int p0 = (int)((long long)o.llen * k / ni);
    const int p1 = (int)((long long)o.llen * (k + 1) / ni);
    for (int r0 = p0; r0 < p1; r0 += HV_Q) {
      constexpr int EPT = HV_Q / TB_BS;
      const int nq = min(HV_Q, p1 - r0);
      int lens[EPT];
      int lsum = 0;
#pragma unroll
      for (int j = 0; j < EPT; j++) {
        const int qk = tid * EPT + j;
        lens[j] = 0;
        if (qk < nq) {
          const Query q = make_query(a, o, o.lbeg + r0 + qk);
          sh.h.qbeg[qk] = q.beg;
          sh.h.qW[qk] = q.W;
          sh.h.qeid[qk] = q.eid;
          sh.h.qother[qk] = q.other;
          lens[j] = q.len;
        }
        lsum += lens[j];
      }
      int tot;
      int run = block_excl_scan<TB_BS>(lsum, s_ws, &tot);
#pragma unroll
      for (int j = 0; j < EPT; j++) {
        const int qk = tid * EPT + j;
        if (qk < nq) sh.h.qoff[qk] = run;
        run += lens[j];
      }
      if (tid == 0) sh.h.qoff[nq] = tot;
      __syncthreads();
      int hint = 0;
      for (int idx = tid; idx < tot; idx += TB_BS) {
        int qlo = hint, step = 1;  // last q with qoff[q] <= idx
        while (qlo + step < nq && sh.h.qoff[qlo + step] <= idx) {
          qlo += step;
          step <<= 1;
        }
        int qhi = min(qlo + step, nq) - 1;
        while (qlo < qhi) {
          const int mid = (qlo + qhi + 1) >> 1;
          if (sh.h.qoff[mid] <= idx) qlo = mid;
          else qhi = mid - 1;
        }
        hint = qlo;
        const int f = sh.h.qbeg[qlo] + (idx - sh.h.qoff[qlo]);
        int y;
        uint32_t wa;
        if (!scan_elem(a, o, sh.h.qother[qlo], f, y, wa)) continue;
        const uint32_t wb = tb_probe(tkey, tval, tmask, tbits, y);
        if (wb != VAL_INF && Tri<WT>::lt(wa, wb, sh.h.qW[qlo])) a.keep[sh.h.qeid[qlo]] = 0;
      }
      probes += tid == 0 ? (unsigned long long)tot : 0ull;
      __syncthreads();
    }
  }

  // -------------------------------------------- light owners, one per wave
  int32_t *key = sh.l.key[wid];
  uint32_t *val = sh.l.val[wid];
  for (;;) {
    int i0 = 0;
    if (lane == 0) i0 = atomicAdd(&a.tickets[1], WAVE);
    i0 = __shfl(i0, 0, WAVE);
    if (i0 >= 2 * a.n) break;
    const int i1 = min(2 * a.n, i0 + WAVE);
    for (int i = i0; i < i1; i++) {
      if (a.hflag[i] || a.work[i] == 0) continue;
      const Owner o = make_owner(a, i);
      const int tbits = tb_bits(o.llen, 5);
      const int tmask = (1 << tbits) - 1;
      for (int s = lane; s < (1 << tbits); s += WAVE) {
        key[s] = -1;
        val[s] = VAL_INF;
      }
      wave_sync();
      for (int p = lane; p < o.llen; p += WAVE) {
        uint32_t v;
        const int y = list_key(a, o, o.lbeg + p, v);
        if (y >= 0) tb_insert(key, val, tmask, tbits, y, v);
      }
      wave_sync();
      for (int r0 = 0; r0 < o.llen; r0 += WAVE) {
        const int nq = min(WAVE, o.llen - r0);
        int len = 0;
        if (lane < nq) {
          const Query q = make_query(a, o, o.lbeg + r0 + lane);
          sh.l.qbeg[wid][lane] = q.beg;
          sh.l.qW[wid][lane] = q.W;
          sh.l.qeid[wid][lane] = q.eid;
          sh.l.qother[wid][lane] = q.other;
          len = q.len;
        }
        const int incl = wave_incl_scan(len);
        sh.l.qoff[wid][lane] = incl - len;
        const int tot = __shfl(incl, WAVE - 1, WAVE);
        if (lane == 0) sh.l.qoff[wid][nq] = tot;
        wave_sync();
        int hint = 0;
        for (int idx = lane; idx < tot; idx += WAVE) {
          int qlo = hint, step = 1;
          while (qlo + step < nq && sh.l.qoff[wid][qlo + step] <= idx) {
            qlo += step;
            step <<= 1;
          }
          int qhi = min(qlo + step, nq) - 1;
          while (qlo < qhi) {
            const int mid = (qlo + qhi + 1) >> 1;
            if (sh.l.qoff[wid][mid] <= idx) qlo = mid;
            else qhi = mid - 1;
          }
          hint = qlo;
          const int f = sh.l.qbeg[wid][qlo] + (idx - sh.l.qoff[wid][qlo]);
          int y;
          uint32_t wa;
          if (!scan_elem(a, o, sh.l.qother[wid][qlo], f, y, wa)) continue;
          const uint32_t wb = tb_probe(key, val, tmask, tbits, y);
          if (wb != VAL_INF && Tri<WT>::lt(wa, wb, sh.l.qW[wid][qlo]))
            a.keep[sh.l.qeid[wid][qlo]] = 0;
        }
        probes += lane == 0 ? (unsigned long long)tot : 0ull;
        wave_sync();
      }
    }
  }
  if (a.stats) {
    probes = wave_sum(probes);
    if (lane == 0 && probes) stat_add(&a.stats->wedges, probes);
  }
}

__global__ void k_tb_count_pruned(const uint8_t *keep, int m, sssp_stats *stats,
                                  const int32_t *status) {
  if (*status || !stats) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  unsigned int c = 0;
  for (int e = t; e < m; e += stride) c += keep[e] == 0;
  c = wave_sum(c);
  if (lane_id() == 0 && c) stat_add(&stats->edges_pruned, c);
}

// ------------------------------------------------------------ compaction
// pos = exclusive scan of keep over all arcs: kept arc e goes to pos[e], and
// the pruned row u starts at pos[row_ptr[u]] (order is preserved).
__global__ void k_compact(const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                          const uint8_t *keep, int n, int m, const int32_t *pos,
                          int32_t *out_row_ptr, int32_t *out_col, uint32_t *out_w,
                          int32_t *edge_map, const int32_t *status) {
  if (*status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < m; e += stride)
    if (keep[e]) {
      const int p = pos[e];
      out_col[p] = col[e];
      out_w[p] = w[e];
      edge_map[p] = e;
    }
  for (int u = t; u <= n; u += stride) out_row_ptr[u] = pos[row_ptr[u]];
}

// ------------------------------------------------------------ host side
namespace {
struct PruneLayout {
  int rep;
  size_t src, cnt, cptr, cursor, cyw, ceid, ryw, work, hflag, hpos, hid, hitems, hoff, gsz,
      goff, gkey, gval, tmp, misc, pos, total;
};

int replicas(int n) {
  if ((long long)n * 16 <= (1ll << 26)) return 16;
  if ((long long)n * 4 <= (1ll << 28)) return 4;
  return 1;
}

PruneLayout prune_layout(int n, int m, bool compact) {
  PruneLayout L;
  size_t off = 0;
  auto take = [&](size_t x) {
    const size_t at = off;
    off += align_up(x ? x : 1, 256);
    return at;
  };
  L.rep = replicas(n);
  const size_t n2 = 2ull * n;
  const size_t nr = (size_t)n * L.rep;
  // the global tables hold at most 2 slots per list entry, rounded up to a
  // power of two: below 8 m slots over all in- and out-lists
  const size_t gslots = 8ull * (size_t)m + G_UNIT;
  L.src = take(4ull * m);
  L.cnt = take(4 * nr);
  L.cptr = take(4 * (nr + 1));
  L.cursor = take(4 * nr);
  L.cyw = take(8ull * m);
  L.ceid = take(4ull * m);
  L.ryw = take(8ull * m);
  L.work = take(4 * n2);
  L.hflag = take(4 * n2);
  L.hpos = take(4 * (n2 + 1));
  L.hid = take(4 * n2);
  L.hitems = take(4 * n2);
  L.hoff = take(4 * (n2 + 1));
  L.gsz = take(4 * n2);
  L.goff = take(4 * (n2 + 1));
  L.gkey = take(4 * gslots);
  L.gval = take(4 * gslots);
  const size_t scan_n = nr > n2 + 1 ? nr : n2 + 1;
  L.tmp = take(scan_tmp_bytes((int)(scan_n > (size_t)m + 1 ? scan_n : (size_t)m + 1)));
  L.misc = take(256);
  L.pos = compact ? take(4ull * (m + 1)) : 0;
  L.total = off;
  return L;
}
}  // namespace

size_t prune_ws_bytes(int n, int m, bool compact) { return prune_layout(n, m, compact).total; }

int launch_prune(const sssp_csr &g, int local, int bsize, uint8_t *keep, int32_t *out_row_ptr,
                 int32_t *out_col, void *out_w, int32_t *edge_map, sssp_stats *stats,
                 char *ws, int grid_cus, bool validate, void *ev_start, void *ev_stop,
                 int32_t **status_out, hipStream_t st) {
  const int n = g.n, m = g.m;
  const PruneLayout L = prune_layout(n, m, out_row_ptr != nullptr);
  TbArgs a;
  a.row_ptr = g.row_ptr;
  a.col = g.col;
  a.w = static_cast<const uint32_t *>(g.w);
  a.n = n;
  a.m = m;
  a.local = local;
  a.bsize = bsize;
  a.keep = keep;
  a.rep = L.rep;
  a.src = reinterpret_cast<int32_t *>(ws + L.src);
  a.cnt = reinterpret_cast<int32_t *>(ws + L.cnt);
  a.cptr = reinterpret_cast<int32_t *>(ws + L.cptr);
  a.cursor = reinterpret_cast<int32_t *>(ws + L.cursor);
  a.cyw = reinterpret_cast<int2 *>(ws + L.cyw);
  a.ceid = reinterpret_cast<int32_t *>(ws + L.ceid);
  a.ryw = reinterpret_cast<int2 *>(ws + L.ryw);
  a.work = reinterpret_cast<int32_t *>(ws + L.work);
  a.hflag = reinterpret_cast<int32_t *>(ws + L.hflag);
  a.hpos = reinterpret_cast<int32_t *>(ws + L.hpos);
  a.hid = reinterpret_cast<int32_t *>(ws + L.hid);
  a.hitems = reinterpret_cast<int32_t *>(ws + L.hitems);
  a.hoff = reinterpret_cast<int32_t *>(ws + L.hoff);
  a.gsz = reinterpret_cast<int32_t *>(ws + L.gsz);
  a.goff = reinterpret_cast<int32_t *>(ws + L.goff);
  a.gkey = reinterpret_cast<int32_t *>(ws + L.gkey);
  a.gval = reinterpret_cast<uint32_t *>(ws + L.gval);
  int32_t *tmp = reinterpret_cast<int32_t *>(ws + L.tmp);
  char *misc = ws + L.misc;
  a.tickets = reinterpret_cast<int32_t *>(misc);
  a.status = reinterpret_cast<int32_t *>(misc + 16);
  a.stats = stats;
  int32_t *pos = out_row_ptr ? reinterpret_cast<int32_t *>(ws + L.pos) : nullptr;
  *status_out = a.status;

  const int blocks = 2048;
  hipLaunchKernelGGL(k_tb_status, dim3(1), dim3(64), 0, st, a);
  if (validate && launch_validate(g, 1, 0, a.status, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tb_zero, dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_tb_tails, dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_tb_indeg, dim3(blocks), dim3(256), 0, st, a);
  if (launch_excl_scan(a.cnt, n * L.rep, a.cptr, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tb_fill, dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_tb_work, dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_tb_classify, dim3(blocks), dim3(256), 0, st, a);
  if (launch_excl_scan(a.hflag, 2 * n, a.hpos, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
  if (launch_excl_scan(a.gsz, 2 * n, a.goff, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tb_heavy_list, dim3(blocks), dim3(256), 0, st, a);
  if (launch_excl_scan(a.hitems, 2 * n, a.hoff, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tb_gtab, dim3(grid_cus * 4), dim3(256), 0, st, a);
  int per_cu = 0;
  if (ev_start && hipEventRecord((hipEvent_t)ev_start, st) != hipSuccess) return SSSP_ERR_HIP;
  if (g.wtype == SSSP_W_U32) {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tb_main<SSSP_W_U32>, TB_BS, 0);
    hipLaunchKernelGGL(k_tb_main<SSSP_W_U32>, dim3(grid_cus * (per_cu > 0 ? per_cu : 1)),
                       dim3(TB_BS), 0, st, a);
  } else {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tb_main<SSSP_W_F32>, TB_BS, 0);
    hipLaunchKernelGGL(k_tb_main<SSSP_W_F32>, dim3(grid_cus * (per_cu > 0 ? per_cu : 1)),
                       dim3(TB_BS), 0, st, a);
  }
  if (hipGetLastError() != hipSuccess) return SSSP_ERR_HIP;
  if (ev_stop && hipEventRecord((hipEvent_t)ev_stop, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tb_count_pruned, dim3(512), dim3(256), 0, st, keep, m, stats, a.status);
  if (out_row_ptr) {
    if (launch_excl_scan_u8(keep, m, pos, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(256), 0, st, g.row_ptr, g.col,
                       static_cast<const uint32_t *>(g.w), keep, n, m, pos, out_row_ptr, out_col,
                       static_cast<uint32_t *>(out_w), edge_map, a.status);
  }
  hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st, a.status, stats);
  return hipGetLastError() == hipSuccess ? SSSP_OK : SSSP_ERR_HIP;
}

}  // namespace sssp_impl
