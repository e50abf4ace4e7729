// prune.hip -- Trishla triangle pruning (Sec. III-B, Alg. 1) on gfx950.
//
// Arc e = (u,x,W) is deleted when some middle y, y != u and y != x, has arcs
// (u,y,w1) and (y,x,w2) with w1 + w2 < W, tested against the input graph for
// all arcs at once.  The middles of e are N_out(u) intersected with N_in(x).
//
// Edge-centric form: for every arc the shorter of the two lists is scanned
// and every entry probed in a hash table of the longer one (keyed by the
// middle vertex, holding the cheapest parallel arc).  The work is at most
// sum_e min(|N_out(u)|, |N_in(x)|) probes instead of the
// sum_y indeg(y) * outdeg(y) wedges of the literal per-vertex loop, and
// far less in practice:
//
//  * every list of SORT_MIN+1 .. SORT_MAX entries is sorted by cost, so the
//    scan of an arc of cost W stops at the first entry with cost >= W (no
//    later entry can be the cheap half of a detour), and
//  * the scan of an arc stops at its first witness.
//
// The scans advance in rounds: each live arc takes a chunk of its list
// (Q_D0 entries, doubling every round), the chunks of all live arcs are
// laid end to end over the lanes, and a finished arc's slot takes the next
// arc of the work item (one wave per light owner: batches of 64 arcs).
//
//  * arcs with |N_out(u)| <= |N_in(x)| ("x-side") are grouped by x and use
//    the table of N_in(x); the others ("u-side") are grouped by u and use
//    the table of N_out(u);
//  * N_in(x) comes from a CSC (in-lists) built here by a counting sort;
//  * a table owner with a short list and little work is handled by one
//    wavefront with a private LDS table; heavier owners are split into
//    workgroup items of about HV_TARGET estimated probes, in four tiers by
//    list length (LDS tables of 1024, 2048 and 4096 slots for 256-thread
//    workgroups, 16384 slots for 1024-thread workgroups, or an L2-resident
//    global table when the list exceeds HV_TCAP entries), so that short
//    tables leave room for more resident workgroups.
//
// Integer costs are summed in 64 bits; fp32 costs are summed in double,
// which decides w1 + w2 < W exactly for fp32 operands (the sum is exact
// unless one operand is below 2^-29 of the other, and then the comparison
// with an fp32 W cannot flip).
#include <array>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

namespace sssp_impl {

constexpr int TB_BS = 1024;
constexpr int LT_DEG = 128;          // light owner: list length
constexpr int LT_SLOTS = 256;        // light owner: wave-private hash slots
constexpr int LT_WORK = 8192;        // light owner: probes
constexpr int LT_BS = 256;
// heavy tiers by list length: LDS tables of 2x the longest list (load <= 1/2)
constexpr int NTIER = 4;
constexpr int T_BIG = NTIER - 1;      // big owners: 1024-thread items
constexpr int HS_TCAP = 512;          // tier 0: longest list
constexpr int HS_SLOTS = 1024;
constexpr int HM1_TCAP = 1024;        // tier 1
constexpr int HM1_SLOTS = 2048;
constexpr int HM_TCAP = 2048;         // tier 2
constexpr int HM_SLOTS = 4096;
// ticket counters: [0, NTIER) heavy items per tier, then the sort queues
// and the light owners
constexpr int TK_SORT_SHORT = NTIER, TK_SORT_LONG = NTIER + 1, TK_LIGHT = NTIER + 2;
constexpr int HM_BS = 256;
constexpr int HM_Q = 256;            // medium: arcs staged per batch
constexpr int HM_MARKS = 1024;       // medium: slot marks of a round
constexpr int HM_FSH = 3;            // 256-thread tiers: filter bits per table slot, log2
constexpr int HV_TCAP = 8192;        // big heavy owner: longest list in an LDS table
constexpr int HV_SLOTS = 16384;
constexpr int HV_Q = 512;            // big: arcs staged per batch
constexpr int HV_MARKS = 2048;       // big: slot marks of a round
constexpr int HV_FSH = 1;            // big: filter bits per LDS table slot, log2
constexpr int ITEM_MINQ = 32;        // an item covers at least this many arcs
constexpr int HV_TARGET = 1 << 18;   // heavy: estimated probes per item
constexpr int HV_TARGET_BIG = 1 << 20;  // big tier: larger items, fewer table rebuilds
constexpr int SORT_MIN = 16;         // lists of SORT_MIN+1 .. SORT_MAX entries
constexpr int SORT_MAX = 4096;       //   are sorted by cost
constexpr int SORT_WAVE = 4 * 64;    // longest list sorted by one wave
#ifndef SSSP_Q_D0
#define SSSP_Q_D0 16
#endif
constexpr int Q_D0 = SSSP_Q_D0;      // first scan chunk of an arc
constexpr int Q_DMAX = 1024;         // chunk cap
constexpr int G_UNIT = 64;           // global table sizes are multiples of this
constexpr uint32_t VAL_INF = 0xFFFFFFFFu;
// Hub pass: the HUB_K vertices with the most two-arc paths through them
// (the largest min(in-degree, out-degree)) are tried as middles of every
// arc before the scans, from dense per-vertex rows of 8-bit cost codes; an
// arc they delete is not scanned.  Only for integer costs, GLOBAL scope and
// n <= HUB_NMAX (the two code tables take 2 * HUB_K bytes per vertex).
constexpr int HUB_K = 32;
constexpr int HUB_NMAX = 1 << 23;
constexpr int HUB_BINS = 512;         // score histogram: 16 bins per octave
constexpr uint8_t HUB_NONE = 0xFF;    // no hub / no arc
// parameters after the histogram and the hub ids
constexpr int HP_WMIN = 0, HP_WMAX = 1, HP_CNT = 2, HP_CNT_TB = 3, HP_STEP = 4, HP_N = 8;

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

// Heavy owners of one tier, in the order they were appended: the owner
// (id), its item count and the first of its items (off), and the slot of
// the owner of every item (map).
struct HList {
  int32_t *id, *items, *off, *map;
};

struct TbArgs {
  const int32_t *row_ptr;
  const int32_t *col;
  const uint32_t *w;
  int n, m, local, bsize;
  uint8_t *keep;
  int cs, nb;       // CSC build: buckets of heads x >> cs, nb of them
  int ct;           // CSC build: arcs per tile
  int32_t *src;     // m: tail of every arc
  int32_t *trow;    // m / TL_E + 1: row of the first arc of every tail tile
  int32_t *btot;    // nb: arcs per bucket
  int32_t *bfill;   // nb: arcs placed per bucket
  int32_t *bstart;  // nb+1: bucket offsets in stage
  int4 *stage;      // m: arcs (x, u, cost, e) grouped by bucket (aliases gkey)
  int32_t *ccnt;    // n: in-degrees
  int32_t *cfill;   // n: CSC entries placed per column
  int32_t *cb;      // n+1: column x is [cb[x], cb[x+1])
  int2 *cyw;        // m: CSC entries (tail, cost); sorted lists by cost
  int32_t *ceid;    // m: CSC -> CSR edge id (moves with cyw)
  int2 *rs;         // m: CSR rows as (head, cost); sorted lists by cost
  int2 *lmeta;      // 2n: (least cost, bucket shift) of an ordered list; shift -1: unordered
  int32_t *sl;      // 2n: lists to sort, short ones from the front, long
                    //     ones (> SORT_WAVE entries) from the back
  int32_t *work;    // 2n: probes of owner i (i < n: in-table of i; else out-table of i-n)
  int32_t *hflag;   // 2n: 0 light or no work, else heavy tier + 1
  HList hl[NTIER];  // heavy owners per tier (T_BIG: the longest lists)
  int32_t *gsz;     // 2n: global table size in units of G_UNIT slots (0 = LDS)
  int32_t *goff;    // 2n: its offset (units), for owners with gsz > 0
  int32_t *hc;      // [t] heavy owners of tier t, [NTIER + t] their items,
                    // [2 NTIER] global table units
  int32_t *gkey;    // global tables: keys (-1 = empty)
  uint32_t *gval;   //                cheapest parallel arc
  int32_t *llist;   // 2n: light owners (order of appending)
  int32_t *tickets; // TK_* counters
  int32_t *status;
  sssp_stats *stats;
  // hub pass (hubs != 0): the HUB_K best middles tried for every scanned arc first
  int hubs;
  uint8_t *hin;     // n x HUB_K: code of the cheapest arc v -> hub k (HUB_NONE = none)
  uint8_t *hout;    // n x HUB_K: code of the cheapest arc hub k -> v
  int32_t *hubm;    // HUB_BINS histogram, HUB_K hub ids, then HP_* parameters
                    // (HP_WMIN / HP_WMAX: least and greatest cost)
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

// Membership filter of a table: one bit per hash of the key (2^fbits bits,
// fbits >= 5), set for every key of the list.  Most probes find their key
// absent; the filter turns those into one LDS word read, so the probe loop,
// whose longest run in a wave holds up every lane, runs only for the few
// lanes that pass.
__device__ __forceinline__ uint32_t tf_hash(int y, int fbits) {
  return ((uint32_t)y * 0x85EBCA6Bu) >> (32 - fbits);
}
__device__ __forceinline__ void tf_set(uint32_t *filt, int fbits, int y) {
  const uint32_t h = tf_hash(y, fbits);
  atomicOr(&filt[h >> 5], 1u << (h & 31));
}
__device__ __forceinline__ bool tf_maybe(const uint32_t *filt, int fbits, int y) {
  const uint32_t h = tf_hash(y, fbits);
  return (filt[h >> 5] >> (h & 31)) & 1u;
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
    for (int k = 0; k <= TK_LIGHT; k++) a.tickets[k] = 0;
    for (int k = 0; k <= 2 * NTIER; k++) a.hc[k] = 0;
  }
  if (a.stats && blockIdx.x == 0 && threadIdx.x < (int)(sizeof(sssp_stats) / 4))
    reinterpret_cast<uint32_t *>(a.stats)[threadIdx.x] = 0u;
}

__device__ __forceinline__ int cbeg(const TbArgs &a, int x) { return a.cb[x]; }
__device__ __forceinline__ int clen(const TbArgs &a, int x) { return a.cb[x + 1] - a.cb[x]; }

__global__ void k_tb_zero(TbArgs a) {
  if (*a.status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < a.m; e += stride) a.keep[e] = 1;
  for (int i = t; i < a.n; i += stride) {
    a.ccnt[i] = 0;
    a.cfill[i] = 0;
  }
  for (int i = t; i < a.nb; i += stride) {
    a.btot[i] = 0;
    a.bfill[i] = 0;
  }
  for (int i = t; i < 2 * a.n; i += stride) a.work[i] = 0;
  if (a.hubs) {
    for (int i = t; i < HUB_BINS; i += stride) a.hubm[i] = 0;
    if (t == 0) {
      a.hubm[HUB_BINS + HUB_K + HP_WMIN] = -1;  // 0xFFFFFFFF as uint32
      a.hubm[HUB_BINS + HUB_K + HP_WMAX] = 0;
      a.hubm[HUB_BINS + HUB_K + HP_CNT] = 0;
      a.hubm[HUB_BINS + HUB_K + HP_CNT_TB] = 0;
    }
  }
}

// Tail of every arc, in tiles of TL_E arcs: k_tb_tilerow records the row
// of every tile's first arc; k_tb_tails stages the bounds of its tile's
// rows in LDS and finds the row of each arc by a binary search there, so
// the stores are coalesced whatever the row lengths.  A tile spanning more
// than TL_ROWS rows (long runs of empty rows) searches row_ptr in place.
constexpr int TL_BS = 256, TL_E = 4096, TL_ROWS = 2048, TL_PT = TL_E / TL_BS;
static_assert(TL_PT % 4 == 0, "whole int4 stores");

__device__ __forceinline__ int tl_tiles(const TbArgs &a) {
  return (int)(((long long)a.m + TL_E - 1) / TL_E);
}

__global__ void k_tb_tilerow(TbArgs a) {
  if (*a.status) return;
  const int nt = tl_tiles(a);
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < a.n; u += gridDim.x * blockDim.x) {
    const int b = a.row_ptr[u], e = a.row_ptr[u + 1];
    for (long long k = ((long long)max(b, 0) + TL_E - 1) / TL_E; k < nt && k * TL_E < e; k++)
      a.trow[k] = u;
  }
}

__global__ __launch_bounds__(TL_BS) void k_tb_tails(TbArgs a) {
  __shared__ int s_rp[TL_ROWS + 1];
  if (*a.status) return;
  const int nt = tl_tiles(a);
  for (int k = blockIdx.x; k < nt; k += gridDim.x) {
    const int e0 = k * TL_E;
    const int e1 = (int)min((long long)a.m, (long long)e0 + TL_E);
    const int u0 = min(max(a.trow[k], 0), a.n - 1);
    const int u1 = k + 1 < nt ? min(max(a.trow[k + 1], u0), a.n - 1) : a.n - 1;
    const int cnt = u1 - u0 + 1;  // rows u0..u1 hold the tile's arcs
    const bool in_lds = cnt <= TL_ROWS;
    if (in_lds)
      for (int r = threadIdx.x; r <= cnt; r += TL_BS) s_rp[r] = a.row_ptr[u0 + r];
    __syncthreads();
    if (in_lds) {
      // TL_PT consecutive arcs per thread: one search for the first, then a
      // walk over the row bounds (at most cnt steps per thread)
      const int ea = e0 + threadIdx.x * TL_PT;
      if (ea < e1) {
        int lo = 0, hi = cnt - 1;  // last row r with row_ptr[u0 + r] <= ea
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_rp[mid] <= ea) lo = mid;
          else hi = mid - 1;
        }
        int out[TL_PT];
#pragma unroll
        for (int i = 0; i < TL_PT; i++) {
          while (lo + 1 < cnt && s_rp[lo + 1] <= ea + i) lo++;
          out[i] = u0 + lo;
        }
        if (ea + TL_PT <= e1) {
          int4 *d = reinterpret_cast<int4 *>(a.src + ea);
#pragma unroll
          for (int i = 0; i < TL_PT / 4; i++)
            d[i] = make_int4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
        } else {
#pragma unroll
          for (int i = 0; i < TL_PT; i++)
            if (ea + i < e1) a.src[ea + i] = out[i];
        }
      }
    } else {
      for (int e = e0 + threadIdx.x; e < e1; e += TL_BS) {
        int lo = 0, hi = cnt - 1;  // last row r with row_ptr[u0 + r] <= e
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (a.row_ptr[u0 + mid] <= e) lo = mid;
          else hi = mid - 1;
        }
        a.src[e] = u0 + lo;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ hubs
// Hub pass.  Most deleted arcs have a witness through one of a few
// high-degree middles (on R-MAT 20, 59% of them through the 32 vertices
// with the most two-arc paths), which a scan reaches only after the
// cheaper entries of its list.  So every arc about to be scanned first
// tries those HUB_K middles at once: row u of `hin` holds the code of the
// cheapest arc u -> hub k, row x of `hout` the code of the cheapest arc
// hub k -> x (HUB_NONE when there is none, and always for a hub's own
// entry in its own rows, since the middle must differ from u and x), and
// the arc is deleted, and not scanned, when some k has both arcs with a
// sum below W.  Codes are upper bounds of the costs, lo + code * step >=
// cost (exact when the costs span at most 254), so every arc deleted this
// way is in the deletion set; any other arc is scanned as before, and the
// result is the same.

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const T y = __shfl_xor(x, o, WAVE);
    x = y > x ? y : x;
  }
  return x;
}

__device__ __forceinline__ uint32_t *hub_params(const TbArgs &a) {
  return reinterpret_cast<uint32_t *>(a.hubm + HUB_BINS + HUB_K);
}

// Score of v as a middle (its two-arc paths are at least score^2; 0 = it
// cannot be one) and its histogram bin (16 bins per octave, monotone).
__device__ __forceinline__ int hub_score(const TbArgs &a, int v) {
  const int od = a.row_ptr[v + 1] - a.row_ptr[v], id = a.ccnt[v];
  return od < id ? od : id;
}
__device__ __forceinline__ int hub_bin(int s) {
  return (int)((__float_as_uint((float)s) - 0x3F800000u) >> 19);
}

// Pass 1: score histogram.  Lanes of a wave with equal bins add once.
__global__ __launch_bounds__(256) void k_hub_hist(TbArgs a) {
  __shared__ int s_h[HUB_BINS];
  if (*a.status) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < HUB_BINS; i += 256) s_h[i] = 0;
  __syncthreads();
  const int t = blockIdx.x * 256 + tid;
  const int stride = gridDim.x * 256;
  const int nr = (a.n + WAVE - 1) / WAVE * WAVE;  // whole waves stay in the loop
  for (int v = t; v < nr; v += stride) {
    int b = -1;
    if (v < a.n) {
      const int sc = hub_score(a, v);
      if (sc > 0) b = hub_bin(sc);
    }
    // one add per distinct bin of the wave
    unsigned long long left = __ballot(b >= 0);
    while (left) {
      const int lead = __ffsll((long long)left) - 1;
      const int bl = __shfl(b, lead, WAVE);
      const unsigned long long same = __ballot(b == bl) & left;
      if (lane_id() == lead) atomicAdd(&s_h[bl], __popcll(same));
      left &= ~same;
    }
  }
  __syncthreads();
  for (int i = tid; i < HUB_BINS; i += 256)
    if (s_h[i]) atomicAdd(&a.hubm[i], s_h[i]);
}

// Pass 2: the hub list; every vertex's two code rows start empty.  Each
// workgroup first finds the threshold bin (every vertex above it is a hub,
// and the first `need` of its own) from the histogram.
__global__ __launch_bounds__(256) void k_hub_take(TbArgs a) {
  __shared__ int s_suf[HUB_BINS + 1];  // vertices in bins >= b
  __shared__ int s_ws[256 / WAVE + 1];
  __shared__ int s_tb, s_need;
  if (*a.status) return;
  uint32_t *hp = hub_params(a);
  {
    // suffix sums of the histogram: two bins per thread, reversed scan
    constexpr int PER = HUB_BINS / 256;
    static_assert(HUB_BINS % 256 == 0, "bins per thread");
    int c[PER], sum = 0;
#pragma unroll
    for (int j = 0; j < PER; j++) {
      c[j] = a.hubm[HUB_BINS - 1 - (threadIdx.x * PER + j)];
      sum += c[j];
    }
    int tot;
    int run = block_excl_scan1<256>(sum, s_ws, &tot);
#pragma unroll
    for (int j = 0; j < PER; j++) {
      run += c[j];
      s_suf[HUB_BINS - 1 - (threadIdx.x * PER + j)] = run;
    }
    if (threadIdx.x == 0) {
      s_suf[HUB_BINS] = 0;
      s_tb = -1;
      s_need = 0;
    }
    __syncthreads();
    // the highest bin b whose suffix reaches HUB_K (unique: suffixes only
    // grow as b falls)
    for (int b = threadIdx.x; b < HUB_BINS; b += 256)
      if (s_suf[b] >= HUB_K && s_suf[b + 1] < HUB_K) {
        s_tb = b;
        s_need = HUB_K - s_suf[b + 1];
      }
    __syncthreads();
  }
  const int tb = s_tb, need = s_need;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t lo = hp[HP_WMIN], hi = hp[HP_WMAX];
    const uint32_t span = hi >= lo ? hi - lo : 0u;
    const uint32_t step = (uint32_t)(((unsigned long long)span + 253ull) / 254ull);
    hp[HP_STEP] = step > 0u ? step : 1u;
  }
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int stride = gridDim.x * 256;
  const int4 none = make_int4(-1, -1, -1, -1);
  for (int v = t; v < a.n; v += stride) {
    const int sc = hub_score(a, v);
    if (sc > 0) {
      const int b = hub_bin(sc);
      if (b > tb || (b == tb && (int)atomicAdd(&hp[HP_CNT_TB], 1u) < need)) {
        const int idx = (int)atomicAdd(&hp[HP_CNT], 1u);  // at most HUB_K in all
        if (idx < HUB_K) a.hubm[HUB_BINS + idx] = v;
      }
    }
    int4 *ri = reinterpret_cast<int4 *>(a.hin + (size_t)v * HUB_K);
    int4 *ro = reinterpret_cast<int4 *>(a.hout + (size_t)v * HUB_K);
#pragma unroll
    for (int k = 0; k < HUB_K / 16; k++) {
      ri[k] = none;
      ro[k] = none;
    }
  }
}

// Code of cost c: the least code whose value lo + code * step is >= c.
__device__ __forceinline__ uint32_t hub_code(uint32_t c, uint32_t lo, uint32_t step) {
  return (uint32_t)(((unsigned long long)(c - lo) + step - 1ull) / step);
}

// Pass 3 (blockIdx.y = hub k): the code rows from hub k's out-row (arcs
// k -> x into hout) and in-column (arcs u -> k into hin); self-loops are
// never a middle's arc.  Plain byte stores: where parallel arcs make two
// stores to one byte, whichever lands is the code of one of those arcs,
// still an upper bound of the cheapest (the row is sorted, so out-row runs
// store the cheapest of the run).
__global__ __launch_bounds__(256) void k_hub_tables(TbArgs a) {
  if (*a.status) return;
  const uint32_t *hp = hub_params(a);
  const int k = blockIdx.y;
  if (k >= (int)min(hp[HP_CNT], (uint32_t)HUB_K)) return;
  const uint32_t lo = hp[HP_WMIN], step = hp[HP_STEP];
  const int h = a.hubm[HUB_BINS + k];
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int stride = gridDim.x * 256;
  const int r0 = a.row_ptr[h], r1 = a.row_ptr[h + 1];
  for (int p = r0 + t; p < r1; p += stride) {
    const int x = a.col[p];
    if (x == h || (unsigned)x >= (unsigned)a.n || (p > r0 && a.col[p - 1] == x)) continue;
    uint32_t c = a.w[p];
    for (int q = p + 1; q < r1 && a.col[q] == x; q++) c = min(c, a.w[q]);  // a run of parallel arcs
    a.hout[(size_t)x * HUB_K + k] = (uint8_t)hub_code(c, lo, step);
  }
  const int c0 = a.cb[h], c1 = a.cb[h + 1];
  for (int p = c0 + t; p < c1; p += stride) {
    const int2 uw = a.cyw[p];
    if (uw.x != h && (unsigned)uw.x < (unsigned)a.n)
      a.hin[(size_t)uw.x * HUB_K + k] = (uint8_t)hub_code((uint32_t)uw.y, lo, step);
  }
}

// Least code sum over the byte lanes of two words (an absent code, 255,
// makes a sum of at least 255, which never passes the test below).
__device__ __forceinline__ uint32_t min_code_sum(uint32_t p, uint32_t q) {
  const uint32_t s0 = (p & 0x00FF00FFu) + (q & 0x00FF00FFu);
  const uint32_t s1 = ((p >> 8) & 0x00FF00FFu) + ((q >> 8) & 0x00FF00FFu);
  const uint32_t a0 = s0 & 0xFFFFu, a1 = s0 >> 16, b0 = s1 & 0xFFFFu, b1 = s1 >> 16;
  const uint32_t m0 = a0 < a1 ? a0 : a1, m1 = b0 < b1 ? b0 : b1;
  return m0 < m1 ? m0 : m1;
}

// Does some hub middle delete arc (u, x, W)?  (lo + c1 step) + (lo + c2
// step) < W with c1 + c2 the least code sum.
__device__ __forceinline__ bool hub_witness(const TbArgs &a, int u, int x, uint32_t W) {
  const uint32_t *hp = hub_params(a);
  const unsigned long long lo2 = 2ull * hp[HP_WMIN], step = hp[HP_STEP];
  if ((unsigned long long)W <= lo2) return false;
  const uint4 *ri = reinterpret_cast<const uint4 *>(a.hin + (size_t)u * HUB_K);
  const uint4 *ro = reinterpret_cast<const uint4 *>(a.hout + (size_t)x * HUB_K);
  uint4 p[HUB_K / 16], q[HUB_K / 16];
#pragma unroll
  for (int k = 0; k < HUB_K / 16; k++) {
    p[k] = ri[k];
    q[k] = ro[k];
  }
  uint32_t best = 0xFFFFu;
#pragma unroll
  for (int k = 0; k < HUB_K / 16; k++) {
    best = min(best, min_code_sum(p[k].x, q[k].x));
    best = min(best, min_code_sum(p[k].y, q[k].y));
    best = min(best, min_code_sum(p[k].z, q[k].z));
    best = min(best, min_code_sum(p[k].w, q[k].w));
  }
  return lo2 + (unsigned long long)best * step < (unsigned long long)W;
}

// ------------------------------------------------------------------ CSC
// The in-lists come from a two-level counting sort of the arcs by head x,
// built so that almost every atomic lands in LDS:
//  * level 1 groups the arcs by bucket x >> cs (at most CB_MAX buckets) in
//    a staging array: a tile of ct arcs counts its buckets in LDS and
//    reserves its run of every nonempty bucket with one global atomic;
//  * level 2 takes the staged arcs in chunks of CCH.  A chunk holds a short
//    run of buckets, so its heads fall in a window of CW columns (counted in
//    LDS) but for a few in sparse regions (one global atomic each).  A
//    first pass adds the chunk's column counts into the in-degrees; after
//    their scan (the column offsets) a second pass reserves the chunk's run
//    of every column and places the entries.
// The order inside a column is arbitrary; columns are sorted by cost later.
constexpr int CB_MAX = 4096;   // level-1 buckets
constexpr int C_BS = 1024;
constexpr int C_TILES = 512;   // level-1 tiles (at most)
constexpr int CCH = 8192;      // level-2 chunk of staged arcs
constexpr int CW = 4096;       // level-2 LDS column window
constexpr int C_U = 4;         // arcs in flight per thread

__device__ __forceinline__ int stage_x(const TbArgs &a, int p) {
  return reinterpret_cast<const int32_t *>(a.stage)[4ll * p];
}

// Level 1, pass 1: bucket sizes (and the head range check).
__global__ __launch_bounds__(C_BS) void k_csc_hist(TbArgs a) {
  __shared__ int s_h[CB_MAX];
  if (*a.status) return;
  for (int b = threadIdx.x; b < a.nb; b += C_BS) s_h[b] = 0;
  __syncthreads();
  const int e0 = blockIdx.x * a.ct;
  const int e1 = (int)min((long long)a.m, (long long)e0 + a.ct);
  for (int e = e0 + threadIdx.x; e < e1; e += C_BS) {
    const int x = a.col[e];
    if ((unsigned)x < (unsigned)a.n) atomicAdd(&s_h[x >> a.cs], 1);
    else set_status(a.status, SSSP_ERR_CSR);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < a.nb; b += C_BS)
    if (s_h[b]) atomicAdd(&a.btot[b], s_h[b]);
}

// Level 1, pass 2: reserve the tile's run of every bucket, stage the arcs,
// and copy the rows as (head, cost).
__global__ __launch_bounds__(C_BS) void k_csc_scatter(TbArgs a) {
  __shared__ int s_h[CB_MAX];
  if (*a.status) return;
  for (int b = threadIdx.x; b < a.nb; b += C_BS) s_h[b] = 0;
  __syncthreads();
  const int e0 = blockIdx.x * a.ct;
  const int e1 = (int)min((long long)a.m, (long long)e0 + a.ct);
  for (int e = e0 + threadIdx.x; e < e1; e += C_BS) atomicAdd(&s_h[a.col[e] >> a.cs], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < a.nb; b += C_BS)
    if (s_h[b]) s_h[b] = a.bstart[b] + atomicAdd(&a.bfill[b], s_h[b]);
  __syncthreads();
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;  // cost range (for the hub pass's codes)
  for (int e = e0 + threadIdx.x; e < e1; e += C_U * C_BS) {
    int x[C_U], u[C_U], wv[C_U];
#pragma unroll
    for (int k = 0; k < C_U; k++) {  // C_U arcs in flight per thread
      const int ek = e + k * C_BS;
      if (ek < e1) {
        x[k] = a.col[ek];
        u[k] = a.src[ek];
        wv[k] = (int)a.w[ek];
      }
    }
#pragma unroll
    for (int k = 0; k < C_U; k++) {
      const int ek = e + k * C_BS;
      if (ek < e1) {
        a.rs[ek] = make_int2(x[k], wv[k]);
        a.stage[atomicAdd(&s_h[x[k] >> a.cs], 1)] = make_int4(x[k], u[k], wv[k], ek);
        lo = min(lo, (uint32_t)wv[k]);
        hi = max(hi, (uint32_t)wv[k]);
      }
    }
  }
  if (a.hubs) {  // one global atomic pair per workgroup
    lo = wave_min(lo);
    hi = wave_max(hi);
    __syncthreads();  // s_h is free again
    uint32_t *s_r = reinterpret_cast<uint32_t *>(s_h);
    if (threadIdx.x == 0) {
      s_r[0] = 0xFFFFFFFFu;
      s_r[1] = 0u;
    }
    __syncthreads();
    if (lane_id() == 0 && lo <= hi) {
      atomicMin(&s_r[0], lo);
      atomicMax(&s_r[1], hi);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_r[0] <= s_r[1]) {
      uint32_t *hp = hub_params(a);
      atomicMin(&hp[HP_WMIN], s_r[0]);
      atomicMax(&hp[HP_WMAX], s_r[1]);
    }
  }
}

__device__ __forceinline__ int chunk_x0(const TbArgs &a, int p0) {
  return (stage_x(a, p0) >> a.cs) << a.cs;
}

// Level 2, pass 1: in-degrees.
__global__ __launch_bounds__(C_BS) void k_csc_count(TbArgs a) {
  __shared__ int s_c[CW];
  if (*a.status) return;
  const int p0 = blockIdx.x * CCH;
  const int p1 = (int)min((long long)a.m, (long long)p0 + CCH);
  const int x0 = chunk_x0(a, p0);
  for (int c = threadIdx.x; c < CW; c += C_BS) s_c[c] = 0;
  __syncthreads();
  for (int p = p0 + threadIdx.x; p < p1; p += C_BS) {
    const int x = stage_x(a, p);
    if (x - x0 < CW) atomicAdd(&s_c[x - x0], 1);
    else atomicAdd(&a.ccnt[x], 1);
  }
  __syncthreads();
  const int cw = min(CW, a.n - x0);
  for (int c = threadIdx.x; c < cw; c += C_BS)
    if (s_c[c]) atomicAdd(&a.ccnt[x0 + c], s_c[c]);
}

// Level 2, pass 2: place the entries at their column offsets, and charge
// the x-side probes of every arc to its column's table owner: an arc
// (u, x) with |N_out(u)| <= |N_in(x)| scans N_out(u).
__global__ __launch_bounds__(C_BS) void k_csc_place(TbArgs a) {
  __shared__ int s_c[CW];  // counts, then cursors
  __shared__ int s_w[CW];  // probes
  if (*a.status) return;
  const int p0 = blockIdx.x * CCH;
  const int p1 = (int)min((long long)a.m, (long long)p0 + CCH);
  const int x0 = chunk_x0(a, p0);
  const int cw = min(CW, a.n - x0);
  for (int c = threadIdx.x; c < CW; c += C_BS) {
    s_c[c] = 0;
    s_w[c] = 0;
  }
  __syncthreads();
  for (int p = p0 + threadIdx.x; p < p1; p += C_BS) {
    const int x = stage_x(a, p);
    if (x - x0 < CW) atomicAdd(&s_c[x - x0], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cw; c += C_BS)
    if (s_c[c]) s_c[c] = a.cb[x0 + c] + atomicAdd(&a.cfill[x0 + c], s_c[c]);
  __syncthreads();
  for (int p = p0 + threadIdx.x; p < p1; p += C_U * C_BS) {
    int4 r[C_U];
    int ou[C_U], ix[C_U];
#pragma unroll
    for (int k = 0; k < C_U; k++)  // C_U entries in flight per thread
      if (p + k * C_BS < p1) r[k] = a.stage[p + k * C_BS];
#pragma unroll
    for (int k = 0; k < C_U; k++)
      if (p + k * C_BS < p1) {
        ou[k] = a.row_ptr[r[k].y + 1] - a.row_ptr[r[k].y];
        ix[k] = a.cb[r[k].x + 1] - a.cb[r[k].x];
      }
#pragma unroll
    for (int k = 0; k < C_U; k++)
      if (p + k * C_BS < p1) {
        const int x = r[k].x;
        const bool win = x - x0 < CW;
        const int pos = win ? atomicAdd(&s_c[x - x0], 1) : a.cb[x] + atomicAdd(&a.cfill[x], 1);
        a.cyw[pos] = make_int2(r[k].y, r[k].z);
        a.ceid[pos] = r[k].w;
        const int val = ou[k] <= ix[k] ? ou[k] : 0;
        if (val) {
          if (win) atomicAdd(&s_w[x - x0], val);
          else atomicAdd(&a.work[x], val);
        }
      }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cw; c += C_BS)
    if (s_w[c]) atomicAdd(&a.work[x0 + c], s_w[c]);
}

// ------------------------------------------------------------------ order
// List i < n is CSR row i (entries in rs), list n + x is CSC column x
// (entries in cyw, with ceid carried along).  Every list of SORT_MIN+1 ..
// SORT_MAX entries is put in cost order by a counting sort over NBK
// buckets of width 2^s above its least cost lo, s the least shift that
// fits its cost span: an exact cost order when the span is below NBK (any
// integer costs up to 255 apart), bucket order otherwise.  Costs compare
// as uint32 bits (nonnegative floats order the same way).  lmeta keeps
// (lo, s) per ordered list for the scans' stop rule; the order of equal
// buckets is arbitrary.
constexpr int NBK = 256;
constexpr int ORD_BS = 256;          // workgroup of a long list (one bucket per thread)
constexpr int ORD_R = SORT_MAX / ORD_BS;

__device__ __forceinline__ bool sorted_len(int len) { return len > SORT_MIN && len <= SORT_MAX; }

__device__ __forceinline__ int bucket_shift(uint32_t span) {
  int s = 0;
  while ((span >> s) >= (uint32_t)NBK) s++;
  return s;
}

struct SortSeg {
  int beg, len;
  bool row;
};

__device__ __forceinline__ SortSeg sort_seg(const TbArgs &a, int i) {
  SortSeg g;
  g.row = i < a.n;
  if (g.row) {
    g.beg = a.row_ptr[i];
    g.len = a.row_ptr[i + 1] - g.beg;
  } else {
    g.beg = cbeg(a, i - a.n);
    g.len = clen(a, i - a.n);
  }
  return g;
}

__device__ __forceinline__ void ord_get(const TbArgs &a, const SortSeg &g, int p, int2 &yw,
                                        int &pay) {
  yw = g.row ? a.rs[p] : a.cyw[p];
  pay = g.row ? 0 : a.ceid[p];
}

__device__ __forceinline__ void ord_put(const TbArgs &a, const SortSeg &g, int p, int2 yw,
                                        int pay) {
  if (g.row) {
    a.rs[p] = yw;
  } else {
    a.cyw[p] = yw;
    a.ceid[p] = pay;
  }
}

// CLS_K lists per thread and pass: queue the lists to order.  A pass
// reserves its queue runs with one atomic per queue, so the whole grid
// takes a few hundred atomics on the two counters instead of one pair per
// 1024 lists.
constexpr int CLS_BS = 1024;
constexpr int CLS_K = 8;
static_assert(CLS_BS * CLS_K < (1 << 16), "two 16-bit counts in one scan");
__global__ __launch_bounds__(CLS_BS) void k_tb_sort_class(TbArgs a) {
  __shared__ int s_ws[CLS_BS / WAVE + 1];
  __shared__ int s_base[2];
  if (*a.status) return;
  const int tid = threadIdx.x;
  const int n2 = 2 * a.n;
  constexpr int SPAN = CLS_BS * CLS_K;
  for (int i0 = blockIdx.x * SPAN; i0 < n2; i0 += gridDim.x * SPAN) {
    uint32_t cls = 0;  // 2 bits per list: 1 = short queue, 2 = long queue
    int cnt = 0;       // short count | long count << 16
#pragma unroll
    for (int k = 0; k < CLS_K; k++) {
      const int i = i0 + k * CLS_BS + tid;
      if (i >= n2) continue;
      const int len = i < a.n ? a.row_ptr[i + 1] - a.row_ptr[i] : clen(a, i - a.n);
      const uint32_t c = sorted_len(len) ? (len > SORT_WAVE ? 2u : 1u) : 0u;
      cls |= c << (2 * k);
      cnt += c == 1u ? 1 : (c == 2u ? 1 << 16 : 0);
      a.lmeta[i] = make_int2(0, -1);  // unordered unless ordered below
    }
    int tot;
    const int pre = block_excl_scan1<CLS_BS>(cnt, s_ws, &tot);
    if (tid < 2) {
      const int t = tid ? tot >> 16 : tot & 0xFFFF;
      s_base[tid] = t ? atomicAdd(&a.tickets[TK_SORT_SHORT + tid], t) : 0;
    }
    __syncthreads();
    int offs = s_base[0] + (pre & 0xFFFF), offl = s_base[1] + (pre >> 16);
#pragma unroll
    for (int k = 0; k < CLS_K; k++) {
      const uint32_t c = (cls >> (2 * k)) & 3u;
      const int i = i0 + k * CLS_BS + tid;
      if (c == 1u) a.sl[offs++] = i;
      else if (c == 2u) a.sl[n2 - 1 - offl++] = i;
    }
    __syncthreads();  // s_ws and s_base are reused by the next pass
  }
}

// One wave per short queued list (SORT_MIN < length <= SORT_WAVE): the
// entries stay in registers, the bucket counters in the wave's LDS.
template <int R>
__device__ __forceinline__ void wave_order(const TbArgs &a, int li, const SortSeg &g, int *cnt) {
  const int lane = lane_id();
  int2 yw[R];
  int pay[R], bk[R], rk[R];
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int e = lane + WAVE * r;
    pay[r] = 0;
    yw[r] = make_int2(0, 0);
    if (e < g.len) {
      ord_get(a, g, g.beg + e, yw[r], pay[r]);
      lo = min(lo, (uint32_t)yw[r].y);
      hi = max(hi, (uint32_t)yw[r].y);
    }
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  const int s = bucket_shift(hi - lo);
  for (int b = lane; b < NBK; b += WAVE) cnt[b] = 0;
  wave_sync();
#pragma unroll
  for (int r = 0; r < R; r++)
    if (lane + WAVE * r < g.len) {
      bk[r] = (int)(((uint32_t)yw[r].y - lo) >> s);
      rk[r] = atomicAdd(&cnt[bk[r]], 1);
    }
  wave_sync();
  // exclusive scan of the NBK counters, NBK / WAVE consecutive ones per lane
  constexpr int PL = NBK / WAVE;
  int c[PL], sum = 0;
#pragma unroll
  for (int k = 0; k < PL; k++) {
    c[k] = cnt[lane * PL + k];
    sum += c[k];
  }
  int off = wave_incl_scan(sum) - sum;
#pragma unroll
  for (int k = 0; k < PL; k++) {
    cnt[lane * PL + k] = off;
    off += c[k];
  }
  wave_sync();
#pragma unroll
  for (int r = 0; r < R; r++)
    if (lane + WAVE * r < g.len) ord_put(a, g, g.beg + cnt[bk[r]] + rk[r], yw[r], pay[r]);
  if (lane == 0) a.lmeta[li] = make_int2((int)lo, s);
  wave_sync();
}

__global__ __launch_bounds__(256) void k_tb_sort_small(TbArgs a) {
  __shared__ int s_cnt[256 / WAVE][NBK];
  if (*a.status) return;
  int *cnt = s_cnt[threadIdx.x / WAVE];
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nwaves = gridDim.x * blockDim.x / WAVE;
  const int ns = a.tickets[TK_SORT_SHORT];
  for (int j = wave; j < ns; j += nwaves) {
    const int li = a.sl[j];
    const SortSeg g = sort_seg(a, li);
    if (g.len <= WAVE) wave_order<1>(a, li, g, cnt);
    else if (g.len <= 2 * WAVE) wave_order<2>(a, li, g, cnt);
    else wave_order<4>(a, li, g, cnt);
  }
}

// One workgroup per long queued list (SORT_WAVE < length <= SORT_MAX):
// ORD_R entries per thread in registers, one bucket counter per thread.
__global__ __launch_bounds__(ORD_BS) void k_tb_sort_mid(TbArgs a) {
  static_assert(ORD_BS == NBK, "one bucket per thread");
  __shared__ int s_cnt[NBK];
  __shared__ uint32_t s_lo[ORD_BS / WAVE], s_hi[ORD_BS / WAVE];
  __shared__ int s_ws[ORD_BS / WAVE + 1];
  if (*a.status) return;
  const int tid = threadIdx.x;
  const int nl = a.tickets[TK_SORT_LONG];
  for (int j = blockIdx.x; j < nl; j += gridDim.x) {
    const int li = a.sl[2 * a.n - 1 - j];
    const SortSeg g = sort_seg(a, li);
    int2 yw[ORD_R];
    int pay[ORD_R], bk[ORD_R], rk[ORD_R];
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
    for (int r = 0; r < ORD_R; r++) {
      const int e = tid + ORD_BS * r;
      pay[r] = 0;
      yw[r] = make_int2(0, 0);
      if (e < g.len) {
        ord_get(a, g, g.beg + e, yw[r], pay[r]);
        lo = min(lo, (uint32_t)yw[r].y);
        hi = max(hi, (uint32_t)yw[r].y);
      }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (lane_id() == 0) {
      s_lo[tid / WAVE] = lo;
      s_hi[tid / WAVE] = hi;
    }
    s_cnt[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < ORD_BS / WAVE; w++) {
      lo = min(lo, s_lo[w]);
      hi = max(hi, s_hi[w]);
    }
    const int s = bucket_shift(hi - lo);
#pragma unroll
    for (int r = 0; r < ORD_R; r++)
      if (tid + ORD_BS * r < g.len) {
        bk[r] = (int)(((uint32_t)yw[r].y - lo) >> s);
        rk[r] = atomicAdd(&s_cnt[bk[r]], 1);
      }
    __syncthreads();
    int tot;
    const int off = block_excl_scan<ORD_BS>(s_cnt[tid], s_ws, &tot);
    s_cnt[tid] = off;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ORD_R; r++)
      if (tid + ORD_BS * r < g.len) ord_put(a, g, g.beg + s_cnt[bk[r]] + rk[r], yw[r], pay[r]);
    if (tid == 0) a.lmeta[li] = make_int2((int)lo, s);
    __syncthreads();
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

// Probes of the u-side arcs, charged to their table owner: an arc (u, x)
// with |N_out(u)| > |N_in(x)| scans N_in(x) against the table of N_out(u),
// owner n+u (one thread per arc; the x-side arcs are charged while the CSC
// is placed).
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
}

__device__ __forceinline__ int owner_len(const TbArgs &a, int i) {
  if (i < a.n) return clen(a, i);
  const int u = i - a.n;
  return a.row_ptr[u + 1] - a.row_ptr[u];
}

// Tier of every owner, CLF_K owners per thread and pass.  Light owners with
// work are appended to llist; heavy owners to their tier's list with their
// items (about HV_TARGET estimated probes each, at least ITEM_MINQ arcs),
// slots and item ranges reserved with one atomic per pass and tier; an
// owner with a global table reserves its slots.
constexpr int CLF_BS = 1024;
constexpr int CLF_K = 4;
__global__ __launch_bounds__(CLF_BS) void k_tb_classify(TbArgs a) {
  __shared__ int s_ws[CLF_BS / WAVE + 1];
  __shared__ int s_base;
  __shared__ int s_h[2 * NTIER];  // owners and items per tier, then their bases
  if (*a.status) return;
  const int tid = threadIdx.x;
  const int n2 = 2 * a.n;
  constexpr int SPAN = CLF_BS * CLF_K;
  for (int i0 = blockIdx.x * SPAN; i0 < n2; i0 += gridDim.x * SPAN) {
    if (tid < 2 * NTIER) s_h[tid] = 0;
    __syncthreads();
    int tier[CLF_K], items[CLF_K], jl[CLF_K], ol[CLF_K];
    uint32_t light = 0, heavy = 0;  // bit k: owner k of this thread
    int nlight = 0;
#pragma unroll
    for (int k = 0; k < CLF_K; k++) {
      const int i = i0 + k * CLF_BS + tid;
      tier[k] = 0;
      items[k] = 0;
      jl[k] = 0;
      ol[k] = 0;
      if (i >= n2) continue;
      const int wk = a.work[i];
      const int len = owner_len(a, i);
      const bool hv = wk > 0 && (len > LT_DEG || wk > LT_WORK);
      const int tr = len > HM_TCAP ? T_BIG : (len > HM1_TCAP ? 2 : (len > HS_TCAP ? 1 : 0));
      if (hv) {
        const int cap = len / ITEM_MINQ > 1 ? len / ITEM_MINQ : 1;
        const long long tgt = tr == T_BIG ? HV_TARGET_BIG : HV_TARGET;
        const long long want = ((long long)wk + tgt - 1) / tgt;
        items[k] = want < 1 ? 1 : (want > cap ? cap : (int)want);
        tier[k] = tr;
        heavy |= 1u << k;
        jl[k] = atomicAdd(&s_h[tr], 1);
        ol[k] = atomicAdd(&s_h[NTIER + tr], items[k]);
      } else if (wk > 0) {
        light |= 1u << k;
        nlight++;
      }
      // hflag = heavy tier + 1 (0 = light or no work)
      a.hflag[i] = hv ? tr + 1 : 0;
      int g = 0;
      if (hv && tr == T_BIG && len > HV_TCAP) g = (1 << tb_bits(len, 6)) / G_UNIT;
      a.gsz[i] = g;
      if (g) a.goff[i] = atomicAdd(&a.hc[2 * NTIER], g);
    }
    // the scan's barrier also completes the tier counts in s_h
    int tot;
    const int pre = block_excl_scan1<CLF_BS>(nlight, s_ws, &tot);
    if (tid == 0) s_base = tot ? atomicAdd(&a.tickets[TK_LIGHT], tot) : 0;
    if (tid < 2 * NTIER) {
      const int v = s_h[tid];
      s_h[tid] = v ? atomicAdd(&a.hc[tid], v) : 0;
    }
    __syncthreads();
    int off = s_base + pre;
#pragma unroll
    for (int k = 0; k < CLF_K; k++) {
      const int i = i0 + k * CLF_BS + tid;
      if (light >> k & 1u) a.llist[off++] = i;
      if (heavy >> k & 1u) {
        const HList &h = a.hl[tier[k]];
        const int jj = s_h[tier[k]] + jl[k], o = s_h[NTIER + tier[k]] + ol[k];
        h.id[jj] = i;
        h.items[jj] = items[k];
        h.off[jj] = o;
        for (int q = 0; q < items[k]; q++) h.map[o + q] = jj;
      }
    }
    __syncthreads();  // s_ws, s_base and s_h are reused by the next pass
  }
}

// Global tables of the longest lists: every slot cleared (grid stride over
// all tables), then the lists inserted with blockIdx.x over the owners and
// blockIdx.y over slices of each list.
__global__ void k_tb_gclear(TbArgs a) {
  if (*a.status) return;
  const long long total = (long long)a.hc[2 * NTIER] * G_UNIT;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long s = t; s < total; s += stride) {
    a.gkey[s] = -1;
    a.gval[s] = VAL_INF;
  }
}

__global__ __launch_bounds__(256) void k_tb_gtab(TbArgs a) {
  if (*a.status) return;
  const HList &h = a.hl[T_BIG];
  const int nh = a.hc[T_BIG];
  for (int j = blockIdx.x; j < nh; j += gridDim.x) {
    const int i = h.id[j];
    const int g = a.gsz[i];
    if (!g) continue;
    const long long base = (long long)a.goff[i] * G_UNIT;
    const int slots = g * G_UNIT;
    const int bits = tb_bits(slots / 2, 6);
    const bool out_list = i >= a.n;
    const int t = out_list ? i - a.n : i;
    const int lb = out_list ? a.row_ptr[t] : cbeg(a, t);
    const int ll = out_list ? a.row_ptr[t + 1] - lb : clen(a, t);
    for (int p = blockIdx.y * blockDim.x + threadIdx.x; p < ll; p += gridDim.y * blockDim.x) {
      const int2 yw = out_list ? a.rs[lb + p] : a.cyw[lb + p];
      if (yw.x != t) tb_insert(a.gkey + base, a.gval + base, slots - 1, bits, yw.x, (uint32_t)yw.y);
    }
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
  const int2 yw = o.mode ? a.rs[p] : a.cyw[p];
  v = (uint32_t)yw.y;
  return yw.x == o.t ? -1 : yw.x;
}

// The arc at position p of the owner's list: the list to scan
// [beg, beg+len) (len = 0 when the arc belongs to the other side), its cost
// W, its id and its other end.
struct Query {
  int beg, len;
  uint32_t W, stop;  // stop: entries of higher cost end the scan
  int eid, other;
  int hub;           // 1: deleted by a hub middle (not scanned)
};

// Stop bound of a scan of a list with metadata lm (its lmeta entry) for an
// arc of cost W.  Only entries of
// cost <= W - 1 (as uint32 bits: the next lower float for fp32) can be the
// cheap half of a detour; in an ordered list every entry after one in a
// higher bucket than W - 1's costs more, so an entry of cost above the last
// cost of that bucket ends the scan.  Unordered lists never stop; a list
// whose least cost is >= W is not scanned at all (len = 0).
__device__ __forceinline__ uint32_t scan_stop(int2 lm, uint32_t W, int &len) {
  if (len == 0 || lm.y < 0) return 0xFFFFFFFFu;
  const uint32_t lo = (uint32_t)lm.x;
  if (W <= lo) {
    len = 0;
    return 0u;
  }
  const unsigned long long last =
      (unsigned long long)lo + (((unsigned long long)(((W - 1u) - lo) >> lm.y) + 1ull) << lm.y) -
      1ull;
  return last >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)last;
}

__device__ __forceinline__ Query make_query(const TbArgs &a, const Owner &o, int p) {
  Query q;
  if (o.mode == 0) {  // arc (u -> x = t): scan N_out(u) when |N_out(u)| <= |N_in(x)|
    const int2 uw = a.cyw[p];
    const int u = uw.x;
    const int rs = a.row_ptr[u], ou = a.row_ptr[u + 1] - rs;
    const int2 lm = a.lmeta[u];  // loaded with the row bounds, not after them
    q.beg = rs;
    q.len = ou <= o.llen ? ou : 0;
    q.W = (uint32_t)uw.y;
    q.eid = a.ceid[p];
    q.other = u;
    q.stop = scan_stop(lm, q.W, q.len);
  } else {  // arc (u = t -> x): scan N_in(x) when |N_in(x)| < |N_out(u)|
    const int x = a.col[p];
    const int cs = cbeg(a, x), ix = clen(a, x);
    const int2 lm = a.lmeta[a.n + x];
    q.beg = cs;
    q.len = o.llen <= ix ? 0 : ix;
    q.W = a.w[p];
    q.eid = p;
    q.other = x;
    q.stop = scan_stop(lm, q.W, q.len);
  }
  // an arc this owner scans tries the hub middles first
  q.hub = 0;
  if (a.hubs && q.len > 0 &&
      hub_witness(a, o.mode == 0 ? q.other : o.t, o.mode == 0 ? o.t : q.other, q.W)) {
    a.keep[q.eid] = 0;
    q.len = 0;
    q.hub = 1;
  }
  return q;
}

// Examines the scanned entry yw (middle y, its cost) at list position f
// for arc eid (cost W, other end `other`): 0 = go on, STEP_STOP = the list
// is sorted and has reached costs >= W at f (entries from f on cannot
// help), STEP_HIT = a witness was found and the arc is marked.
constexpr int STEP_STOP = 1, STEP_HIT = 2;
template <int WT>
__device__ __forceinline__ int tb_check(const TbArgs &a, const Owner &o, int2 yw, int other,
                                        uint32_t stop, uint32_t W, int eid, const int32_t *tkey,
                                        const uint32_t *tval, int tmask, int tbits,
                                        const uint32_t *filt, int fbits) {
  const int y = yw.x;
  const uint32_t wa = (uint32_t)yw.y;
  if (wa > stop) return STEP_STOP;
  if (wa >= W) return 0;  // w1 >= W: no detour through this entry
  const int u = o.mode == 0 ? other : o.t;
  const int x = o.mode == 0 ? o.t : other;
  if (y == u || y == x) return 0;
  if (a.local && y / a.bsize != u / a.bsize) return 0;
  if (!tf_maybe(filt, fbits, y)) return 0;
  const uint32_t wb = tb_probe(tkey, tval, tmask, tbits, y);
  if (wb != VAL_INF && Tri<WT>::lt(wa, wb, W)) {
    a.keep[eid] = 0;
    return STEP_HIT;
  }
  return 0;
}

// A round lays the chunks of its live arcs end to end: live slot s holds
// arc srec[s].x, entries [soff[s], soff[s+1]) (soff[nlive] = total, every
// slot nonempty).  mark[k] is the slot holding entry k << gshift (and the
// mark after the last one is nlive - 1), so the slot of an entry lies
// between two marks: a binary search over a range that is almost always
// one or two slots.
__device__ __forceinline__ int locate(const int32_t *mark, int gshift, const int32_t *soff,
                                      int idx) {
  const int k = idx >> gshift;
  int lo = mark[k], hi = mark[k + 1];
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (soff[mid] <= idx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Mark spacing 2^g: at most nmarks marks, and at most 8 (+1) per arc of a
// round with chunks of up to D entries (one thread writes an arc's marks).
__device__ __forceinline__ int mark_shift(int tot, int nmarks, int D) {
  int g = 0;
  while (((tot - 1) >> g) + 1 > nmarks || (D >> g) > 8) g++;
  return g;
}

// Live slot of arc q (chunk of c > 0 entries at off): its marks.
__device__ __forceinline__ void put_marks(int32_t *mark, int gshift, int slot, int off, int c) {
  for (int k = (off + (1 << gshift) - 1) >> gshift; (k << gshift) < off + c; k++) mark[k] = slot;
}

// Packs a chunk length with a live count for one prefix scan: sums stay
// below 2^31 for at most 1024 arcs of chunks below 2^20 in total.
constexpr int LIVE_SH = 20;
__device__ __forceinline__ int live_pack(int c) { return c > 0 ? (1 << LIVE_SH) | c : 0; }

// Scan limit of an arc in LDS: entries at list positions >= limit are not
// examined.  A cost stop at f lowers it to f (entries before f may still
// hold the witness and are examined), a witness lowers it to -1.
__device__ __forceinline__ int ld_lim(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lower_lim(int32_t *p, int step, int f) {
  if (step) __hip_atomic_fetch_min(p, step == STEP_HIT ? -1 : f, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
}

constexpr int SCAN_U = 4;  // scanned entries loaded ahead per lane

// Examines the flattened entries idx = first, first+step, ... < tot of the
// staged arcs (LDS arrays of one batch): SCAN_U loads in flight per lane.
// The chain of LDS reads ahead of each list load is kept short: the live
// slot (marks and a short search), then its record (arc, list position of
// the slot's first entry); the arc's record (other end, stop bound, W, id)
// and scan limit are read while the load is in flight.  An entry past a
// limit lowered in this round is loaded but not probed.
template <int WT>
__device__ __forceinline__ void scan_entries(const TbArgs &a, const Owner &o, int first,
                                             int step, int tot, const int32_t *mark, int gshift,
                                             const int32_t *soff, const int2 *srec,
                                             int32_t *qlim, const int4 *qrec,
                                             const int32_t *tkey, const uint32_t *tval,
                                             int tmask, int tbits, const uint32_t *filt,
                                             int fbits) {
  const int2 *list = o.mode == 0 ? a.rs : a.cyw;
  for (int base = first; base < tot; base += SCAN_U * step) {
    int q[SCAN_U], f[SCAN_U];
    int2 yw[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; u++) {
      const int idx = base + u * step;
      f[u] = -1;
      q[u] = 0;
      if (idx < tot) {
        const int2 sr = srec[locate(mark, gshift, soff, idx)];
        q[u] = sr.x;
        f[u] = idx + sr.y;
        yw[u] = list[f[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < SCAN_U; u++) {
      if (f[u] < 0 || f[u] >= ld_lim(&qlim[q[u]])) continue;
      const int4 r = qrec[q[u]];
      lower_lim(&qlim[q[u]],
                tb_check<WT>(a, o, yw[u], r.x, (uint32_t)r.y, (uint32_t)r.z, r.w, tkey, tval,
                             tmask, tbits, filt, fbits),
                f[u]);
    }
  }
}

template <int SLOTS, int QN, int NM, int FSH>
struct TbHeavy {
  int32_t key[SLOTS];     // (key and val are contiguous: the filter of a
  uint32_t val[SLOTS];    //  global table uses them)
  uint32_t filt[(SLOTS << FSH) / 32];  // filter of an LDS table: 2^FSH bits per slot
  int4 qrec[QN];        // per arc: other end, stop bound, W, arc id
  int32_t qlim[QN];      // per arc: scan limit
  int32_t soff[QN + 1];  // live slots of the round: entry offsets,
  int2 srec[QN];         //   (arc, list position of entry 0 of the round),
  int32_t mark[NM + 1];  //   and marks
};
constexpr int LT_MARKS = 128;
constexpr int LT_FSH = 3;  // light: filter bits per table slot, log2
struct TbLight {         // one per wave
  int32_t key[LT_SLOTS];
  uint32_t val[LT_SLOTS];
  uint32_t filt[(LT_SLOTS << LT_FSH) / 32];
  int4 qrec[WAVE];
  int32_t qlim[WAVE];
  int32_t soff[WAVE + 1];
  int2 srec[WAVE];
  int32_t mark[LT_MARKS + 1];
};

// Heavy owners of one tier: workgroup items taken from a ticket counter;
// the owner's table is in LDS (SLOTS slots) or, for the longest lists of
// the big tier, in global memory.
template <int WT, int TIER, int BS, int SLOTS, int QN, int NM, int FSH>
__global__ __launch_bounds__(BS) void k_tb_heavy(TbArgs a) {
  static_assert(QN <= BS && QN <= 1024 && (long long)QN * Q_DMAX < (1 << LIVE_SH), "packing");
  __shared__ TbHeavy<SLOTS, QN, NM, FSH> H;
  __shared__ int s_ws[BS / WAVE + 1];
  __shared__ int s_t, s_next, s_cmax[2];
  if (*a.status) return;
  const int tid = threadIdx.x;
  const HList &hl = a.hl[TIER];
  const int total = a.hc[NTIER + TIER];
  unsigned long long probes = 0, hubdel = 0;
  for (;;) {
    if (tid == 0) s_t = atomicAdd(&a.tickets[TIER], 1);
    __syncthreads();
    const int it = s_t;
    __syncthreads();
    if (it >= total) break;
    const int j = hl.map[it];
    const int i = hl.id[j];
    const int k = it - hl.off[j];
    const int ni = hl.items[j];
    const Owner o = make_owner(a, i);
    const int32_t *tkey;
    const uint32_t *tval;
    uint32_t *filt;
    int tbits, fbits;
    if (TIER == T_BIG && a.gsz[i]) {
      // global table: the whole LDS table space holds its filter
      const long long base = (long long)a.goff[i] * G_UNIT;
      tkey = a.gkey + base;
      tval = a.gval + base;
      tbits = tb_bits(a.gsz[i] * G_UNIT / 2, 6);
      filt = reinterpret_cast<uint32_t *>(H.key);
      fbits = 31 - __clz(2 * SLOTS * 32);
      for (int s = tid; s < (1 << (fbits - 5)); s += BS) filt[s] = 0u;
      __syncthreads();
      for (int p = tid; p < o.llen; p += BS) {
        uint32_t v;
        const int y = list_key(a, o, o.lbeg + p, v);
        if (y >= 0) tf_set(filt, fbits, y);
      }
      __syncthreads();
    } else {
      tbits = tb_bits(o.llen, 6);
      filt = H.filt;
      fbits = tbits + FSH;
      for (int s = tid; s < (1 << tbits); s += BS) {
        H.key[s] = -1;
        H.val[s] = VAL_INF;
      }
      for (int s = tid; s < (1 << (fbits - 5)); s += BS) filt[s] = 0u;
      __syncthreads();
      for (int p = tid; p < o.llen; p += BS) {
        uint32_t v;
        const int y = list_key(a, o, o.lbeg + p, v);
        if (y >= 0) {
          tb_insert(H.key, H.val, (1 << tbits) - 1, tbits, y, v);
          tf_set(filt, fbits, y);
        }
      }
      __syncthreads();
      tkey = H.key;
      tval = H.val;
    }
    const int tmask = (1 << tbits) - 1;
    // This item's share of the owner's arcs.  Slot tid (< QN) holds one arc
    // at a time; at the start of every round a slot whose arc is done (or
    // that holds none) takes the next arc of the item, so rounds stay full
    // instead of draining a fixed batch.  Each arc's chunks double from Q_D0.
    const int p0 = (int)((long long)o.llen * k / ni);
    const int p1 = (int)((long long)o.llen * (k + 1) / ni);
    if (tid == 0) {
      s_next = p0;
      s_cmax[0] = 0;
      s_cmax[1] = 0;
    }
    __syncthreads();
    int cur = 0, D = Q_D0;  // this slot's next list position and chunk
    bool has = false;       // this slot holds an arc
    for (int round = 0;; round++) {
      if (tid < QN && (!has || cur >= H.qlim[tid])) {
        const int pos = atomicAdd(&s_next, 1);
        has = pos < p1;
        if (has) {
          const Query q = make_query(a, o, o.lbeg + pos);
          cur = q.beg;
          D = Q_D0;
          H.qlim[tid] = q.beg + q.len;
          H.qrec[tid] = make_int4(q.other, (int)q.stop, (int)q.W, q.eid);
          hubdel += q.hub;
        }
      }
      const int c = has ? max(0, min(D, H.qlim[tid] - cur)) : 0;
      const int cm = wave_max(c);
      if (lane_id() == 0 && cm > 0) atomicMax(&s_cmax[round & 1], cm);
      int packed;
      // one barrier: s_ws is next written after this round's last barrier
      const int run = block_excl_scan1<BS>(live_pack(c), s_ws, &packed);
      const int tot = packed & ((1 << LIVE_SH) - 1);
      if (tot == 0) {
        // every held arc is done: stop once the item has no arc left
        const bool more = s_next < p1;
        if (tid == 0) s_cmax[(round + 1) & 1] = 0;
        __syncthreads();  // s_next is read by all before the next refill
        if (!more) break;
        continue;
      }
      const int gshift = mark_shift(tot, NM, s_cmax[round & 1]);
      if (c > 0) {
        const int sl = run >> LIVE_SH, off = run & ((1 << LIVE_SH) - 1);
        H.srec[sl] = make_int2(tid, cur - off);
        H.soff[sl] = off;
        put_marks(H.mark, gshift, sl, off, c);
      }
      if (tid == 0) {
        H.soff[packed >> LIVE_SH] = tot;
        H.mark[((tot - 1) >> gshift) + 1] = (packed >> LIVE_SH) - 1;
        s_cmax[(round + 1) & 1] = 0;  // the next round's maximum
      }
      __syncthreads();
      scan_entries<WT>(a, o, tid, BS, tot, H.mark, gshift, H.soff, H.srec, H.qlim, H.qrec, tkey,
                       tval, tmask, tbits, filt, fbits);
      probes += tid == 0 ? (unsigned long long)tot : 0ull;
      __syncthreads();
      cur += c;
      D = min(2 * D, Q_DMAX);
    }
    __syncthreads();
  }
  if (a.stats && tid == 0 && probes) stat_add(&a.stats->wedges, probes);
  if (a.stats) {
    hubdel = wave_sum(hubdel);
    if (lane_id() == 0 && hubdel) stat_add(&a.stats->hub_pruned, hubdel);
  }
}

// Light owners: one wave per owner of llist, a private LDS table.
template <int WT>
__global__ __launch_bounds__(LT_BS) void k_tb_light(TbArgs a) {
  __shared__ TbLight sw[LT_BS / WAVE];
  if (*a.status) return;
  const int lane = lane_id();
  TbLight &L = sw[threadIdx.x / WAVE];
  const int gw = (blockIdx.x * LT_BS + threadIdx.x) / WAVE;
  const int nw = gridDim.x * (LT_BS / WAVE);
  unsigned long long probes = 0, hubdel = 0;
  const int nlight = a.tickets[TK_LIGHT];
  for (int j = gw; j < nlight; j += nw) {
    {
      const int i = a.llist[j];
      const Owner o = make_owner(a, i);
      const int tbits = tb_bits(o.llen, 5);
      const int tmask = (1 << tbits) - 1;
      const int fbits = tbits + LT_FSH;
      for (int s = lane; s < (1 << tbits); s += WAVE) {
        L.key[s] = -1;
        L.val[s] = VAL_INF;
      }
      for (int s = lane; s < (1 << (fbits - 5)); s += WAVE) L.filt[s] = 0u;
      wave_sync();
      for (int p = lane; p < o.llen; p += WAVE) {
        uint32_t v;
        const int y = list_key(a, o, o.lbeg + p, v);
        if (y >= 0) {
          tb_insert(L.key, L.val, tmask, tbits, y, v);
          tf_set(L.filt, fbits, y);
        }
      }
      wave_sync();
      for (int r0 = 0; r0 < o.llen; r0 += WAVE) {
        const int nq = min(WAVE, o.llen - r0);
        int mycur = 0;
        if (lane < nq) {
          const Query q = make_query(a, o, o.lbeg + r0 + lane);
          mycur = q.beg;
          L.qlim[lane] = q.beg + q.len;
          L.qrec[lane] = make_int4(q.other, (int)q.stop, (int)q.W, q.eid);
          hubdel += q.hub;
        }
        wave_sync();
        for (int D = Q_D0;; D = min(2 * D, Q_DMAX)) {
          const int c = lane < nq ? max(0, min(D, L.qlim[lane] - mycur)) : 0;
          const int incl = wave_incl_scan(live_pack(c));
          const int packed = __shfl(incl, WAVE - 1, WAVE);
          const int tot = packed & ((1 << LIVE_SH) - 1);
          if (tot == 0) break;
          const int gshift = mark_shift(tot, LT_MARKS, D);
          if (c > 0) {
            const int run = incl - live_pack(c);
            const int sl = run >> LIVE_SH, off = run & ((1 << LIVE_SH) - 1);
            L.srec[sl] = make_int2(lane, mycur - off);
            L.soff[sl] = off;
            put_marks(L.mark, gshift, sl, off, c);
          }
          if (lane == 0) {
            L.soff[packed >> LIVE_SH] = tot;
            L.mark[((tot - 1) >> gshift) + 1] = (packed >> LIVE_SH) - 1;
          }
          wave_sync();
          scan_entries<WT>(a, o, lane, WAVE, tot, L.mark, gshift, L.soff, L.srec, L.qlim, L.qrec,
                           L.key, L.val, tmask, tbits, L.filt, fbits);
          probes += lane == 0 ? (unsigned long long)tot : 0ull;
          wave_sync();
          mycur += c;
        }
      }
    }
  }
  if (a.stats) {
    probes = wave_sum(probes);
    hubdel = wave_sum(hubdel);
    if (lane == 0 && probes) stat_add(&a.stats->wedges, probes);
    if (lane == 0 && hubdel) stat_add(&a.stats->hub_pruned, hubdel);
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
// The kept arcs before arc e: the kept arcs of the tiles before e's tile
// (SCAN_TILE arcs per tile; toff, a scan of the tiles' kept counts), plus
// those of e's tile before e's 32-arc word (kpre), plus those of the word
// before e (kbits, one bit per arc).  Kept arc e goes there, and the pruned
// row u starts at that count for row_ptr[u] (order is preserved).
// kpre[ceil(m/32)] holds the kept total.
constexpr int KT_BS = 256;
constexpr int KT_EPT = SCAN_TILE / KT_BS;
static_assert(KT_EPT == 8, "a thread's flags are one byte of its 32-arc word");

__global__ __launch_bounds__(KT_BS) void k_keep_tiles(const uint8_t *keep, int m,
                                                      uint32_t *kbits, int32_t *kpre,
                                                      int32_t *tile_sum) {
  __shared__ int s_ws[KT_BS / WAVE + 1];
  const int tid = threadIdx.x;
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)tid * KT_EPT;
  uint32_t m8 = 0;  // bit j: arc base + j is kept
  if (base + KT_EPT <= m && (reinterpret_cast<uintptr_t>(keep) & 7u) == 0) {
    const uint2 v = *reinterpret_cast<const uint2 *>(keep + base);
#pragma unroll
    for (int j = 0; j < 4; j++) {
      m8 |= ((v.x >> (8 * j)) & 0xFFu) ? 1u << j : 0u;
      m8 |= ((v.y >> (8 * j)) & 0xFFu) ? 1u << (4 + j) : 0u;
    }
  } else {
#pragma unroll
    for (int j = 0; j < KT_EPT; j++)
      if (base + j < m && keep[base + j]) m8 |= 1u << j;
  }
  int tot;
  const int pre = block_excl_scan1<KT_BS>(__popc(m8), s_ws, &tot);
  uint32_t word = m8 << (8 * (tid & 3));  // four threads make a word
  word |= __shfl_xor(word, 1);
  word |= __shfl_xor(word, 2);
  if ((tid & 3) == 0 && base < m) {
    kbits[base >> 5] = word;
    kpre[base >> 5] = pre;
  }
  if (tid == 0) tile_sum[blockIdx.x] = tot;
}

__device__ __forceinline__ int kept_before(const uint32_t *kbits, const int32_t *kpre,
                                           const int32_t *toff, int m, int e) {
  if (e <= 0) return 0;
  if (e >= m) return kpre[((long long)m + 31) >> 5];
  const int wi = e >> 5;
  return toff[e / SCAN_TILE] + kpre[wi] + __popc(kbits[wi] & ((1u << (e & 31)) - 1u));
}

__global__ void k_compact(const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                          const uint8_t *keep, int n, int m, const uint32_t *kbits,
                          const int32_t *kpre, const int32_t *toff, int32_t *out_row_ptr,
                          int32_t *out_col, uint32_t *out_w, int32_t *edge_map,
                          const int32_t *status) {
  if (*status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int e = t; e < m; e += stride)
    if (keep[e]) {
      const int p = kept_before(kbits, kpre, toff, m, e);
      out_col[p] = col[e];
      out_w[p] = w[e];
      edge_map[p] = e;
    }
  for (int u = t; u <= n; u += stride)
    out_row_ptr[u] = kept_before(kbits, kpre, toff, m, row_ptr[u]);
}

// ------------------------------------------------------------ host side
namespace {
struct PruneLayout {
  int cs, nb, ct, tiles;
  size_t src, trow, btot, bfill, bstart, stage, ccnt, cfill, cb, cyw, ceid, rs, lmeta, sl, llist, work, hflag, hl[NTIER][4], gsz,
      goff, gkey, gval, tmp, misc, kbits, kpre, hin, hout, hubm, total;
};

PruneLayout prune_layout(int n, int m, bool compact) {
  PruneLayout L;
  size_t off = 0;
  auto take = [&](size_t x) {
    const size_t at = off;
    off += align_up(x ? x : 1, 256);
    return at;
  };
  L.cs = 0;
  while (n > 0 && ((n - 1) >> L.cs) + 1 > CB_MAX) L.cs++;
  L.nb = n > 0 ? ((n - 1) >> L.cs) + 1 : 1;
  // tiles of whole multiples of the workgroup, at most C_TILES of them
  const long long per = ((long long)m + C_TILES - 1) / C_TILES;
  L.ct = (int)((per + C_BS - 1) / C_BS * C_BS);
  if (L.ct < 8 * C_BS) L.ct = 8 * C_BS;
  L.tiles = m > 0 ? (int)(((long long)m + L.ct - 1) / L.ct) : 0;
  const size_t n2 = 2ull * n;
  // the global tables hold at most 2 slots per list entry, rounded up to a
  // power of two: below 8 m slots over all in- and out-lists
  const size_t gslots = 8ull * (size_t)m + G_UNIT;
  L.src = take(4ull * m);
  L.trow = take(4ull * ((size_t)m / TL_E + 2));
  L.btot = take(4 * (size_t)L.nb);
  L.bfill = take(4 * (size_t)L.nb);
  L.bstart = take(4 * ((size_t)L.nb + 1));
  L.ccnt = take(4 * (size_t)n);
  L.cfill = take(4 * (size_t)n);
  L.cb = take(4 * ((size_t)n + 1));
  L.cyw = take(8ull * m);
  L.ceid = take(4ull * m);
  L.rs = take(8ull * m);
  L.lmeta = take(8 * n2);
  L.sl = take(4 * n2);
  L.llist = take(4 * n2);
  L.work = take(4 * n2);
  L.hflag = take(4 * n2);
  for (int t = 0; t < NTIER; t++) {
    L.hl[t][0] = take(4 * n2);                           // id
    L.hl[t][1] = take(4 * n2);                           // items
    L.hl[t][2] = take(4 * n2);                           // off
    // map: an owner has at most max(1, len / ITEM_MINQ) items and the lists
    // hold 2m entries in all
    L.hl[t][3] = take(4 * (n2 + 2ull * (size_t)m / ITEM_MINQ + 64));
  }
  L.gsz = take(4 * n2);
  L.goff = take(4 * n2);
  L.gkey = take(4 * gslots);
  L.stage = L.gkey;  // 16 m bytes, dead before the global tables are cleared
  L.gval = take(4 * gslots);
  const size_t scan_n = n2 + 1;
  L.tmp = take(scan_tmp_bytes((int)(scan_n > (size_t)m + 1 ? scan_n : (size_t)m + 1)));
  L.misc = take(256);
  const size_t nw = ((size_t)m + 31) / 32;
  if (n <= HUB_NMAX) {
    L.hin = take((size_t)n * HUB_K);
    L.hout = take((size_t)n * HUB_K);
    L.hubm = take(4 * (HUB_BINS + HUB_K + HP_N));
  } else {
    L.hin = L.hout = L.hubm = 0;
  }
  L.kbits = compact ? take(4 * nw) : 0;
  L.kpre = compact ? take(4 * (nw + 1)) : 0;
  L.total = off;
  return L;
}
}  // namespace

template <typename K>
void launch_resident(K kernel, int bs, int grid_cus, const TbArgs &a, hipStream_t st) {
  int per_cu = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, bs, 0);
  hipLaunchKernelGGL(kernel, dim3(grid_cus * (per_cu > 0 ? per_cu : 1)), dim3(bs), 0, st, a);
}

// Side streams and fork/join events of one device: created on first use
// (default priority, non-blocking streams) and kept for the life of the
// process.  A call holds side_mutex() from its first fork to its last join,
// so each wait pairs with that call's own record.
constexpr int SIDE_STREAMS = 3, SIDE_EVENTS = 8;
struct SideStreams {
  hipStream_t s[SIDE_STREAMS] = {};
  hipEvent_t ev[SIDE_EVENTS] = {};
  bool ready = false;
};

std::mutex &side_mutex() {
  static std::mutex mu;
  return mu;
}

// Caller holds side_mutex().
SideStreams *side_streams() {
  static std::vector<SideStreams> per_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if ((int)per_dev.size() <= dev) per_dev.resize(dev + 1);
  SideStreams &d = per_dev[dev];
  if (!d.ready) {
    for (int i = 0; i < SIDE_STREAMS; i++)
      if (!d.s[i] && hipStreamCreateWithFlags(&d.s[i], hipStreamNonBlocking) != hipSuccess) {
        d.s[i] = nullptr;
        return nullptr;
      }
    for (int i = 0; i < SIDE_EVENTS; i++)
      if (!d.ev[i] && hipEventCreateWithFlags(&d.ev[i], hipEventDisableTiming) != hipSuccess) {
        d.ev[i] = nullptr;
        return nullptr;
      }
    d.ready = true;
  }
  return &d;
}

// The five scan kernels (light owners, four heavy tiers).  Each drains its
// own ticket queue with resident workgroups, so run concurrently they fill
// each other's tails: the tiers with the longest items go to the side
// streams (forked from st with ev[2], joined back with ev[3..5]).  Without
// side streams (stream capture) they run one after another on st.
template <int WT>
hipError_t launch_scan_kernels(const TbArgs &a, int grid_cus, hipStream_t st, SideStreams *d) {
  static_assert(NTIER == 4, "one launch per heavy tier");
  auto k_light = k_tb_light<WT>;
  auto k_t0 = k_tb_heavy<WT, 0, HM_BS, HS_SLOTS, HM_Q, HM_MARKS, HM_FSH>;
  auto k_t1 = k_tb_heavy<WT, 1, HM_BS, HM1_SLOTS, HM_Q, HM_MARKS, HM_FSH>;
  auto k_t2 = k_tb_heavy<WT, 2, HM_BS, HM_SLOTS, HM_Q, HM_MARKS, HM_FSH>;
  auto k_big = k_tb_heavy<WT, T_BIG, TB_BS, HV_SLOTS, HV_Q, HV_MARKS, HV_FSH>;
  if (!d) {
    launch_resident(k_light, LT_BS, grid_cus, a, st);
    launch_resident(k_t0, HM_BS, grid_cus, a, st);
    launch_resident(k_t1, HM_BS, grid_cus, a, st);
    launch_resident(k_t2, HM_BS, grid_cus, a, st);
    launch_resident(k_big, TB_BS, grid_cus, a, st);
    return hipSuccess;
  }
  hipError_t err;
  if ((err = hipEventRecord(d->ev[2], st)) != hipSuccess) return err;
  for (int i = 0; i < SIDE_STREAMS; i++)
    if ((err = hipStreamWaitEvent(d->s[i], d->ev[2], 0)) != hipSuccess) return err;
  launch_resident(k_big, TB_BS, grid_cus, a, d->s[0]);
  launch_resident(k_t2, HM_BS, grid_cus, a, d->s[1]);
  launch_resident(k_t1, HM_BS, grid_cus, a, d->s[2]);
  launch_resident(k_light, LT_BS, grid_cus, a, st);
  launch_resident(k_t0, HM_BS, grid_cus, a, st);
  for (int i = 0; i < SIDE_STREAMS; i++) {
    if ((err = hipEventRecord(d->ev[3 + i], d->s[i])) != hipSuccess) return err;
    if ((err = hipStreamWaitEvent(st, d->ev[3 + i], 0)) != hipSuccess) return err;
  }
  return hipSuccess;
}

size_t prune_ws_bytes(int n, int m, bool compact) { return prune_layout(n, m, compact).total; }

int launch_prune(const sssp_csr &g, int local, bool hubs, int bsize, uint8_t *keep,
                 int32_t *out_row_ptr,
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
  a.cs = L.cs;
  a.nb = L.nb;
  a.ct = L.ct;
  a.src = reinterpret_cast<int32_t *>(ws + L.src);
  a.trow = reinterpret_cast<int32_t *>(ws + L.trow);
  a.btot = reinterpret_cast<int32_t *>(ws + L.btot);
  a.bfill = reinterpret_cast<int32_t *>(ws + L.bfill);
  a.bstart = reinterpret_cast<int32_t *>(ws + L.bstart);
  a.stage = reinterpret_cast<int4 *>(ws + L.stage);
  a.ccnt = reinterpret_cast<int32_t *>(ws + L.ccnt);
  a.cfill = reinterpret_cast<int32_t *>(ws + L.cfill);
  a.cb = reinterpret_cast<int32_t *>(ws + L.cb);
  a.cyw = reinterpret_cast<int2 *>(ws + L.cyw);
  a.ceid = reinterpret_cast<int32_t *>(ws + L.ceid);
  a.rs = reinterpret_cast<int2 *>(ws + L.rs);
  a.lmeta = reinterpret_cast<int2 *>(ws + L.lmeta);
  a.sl = reinterpret_cast<int32_t *>(ws + L.sl);
  a.llist = reinterpret_cast<int32_t *>(ws + L.llist);
  a.work = reinterpret_cast<int32_t *>(ws + L.work);
  a.hflag = reinterpret_cast<int32_t *>(ws + L.hflag);
  for (int t = 0; t < NTIER; t++) {
    HList &h = a.hl[t];
    h.id = reinterpret_cast<int32_t *>(ws + L.hl[t][0]);
    h.items = reinterpret_cast<int32_t *>(ws + L.hl[t][1]);
    h.off = reinterpret_cast<int32_t *>(ws + L.hl[t][2]);
    h.map = reinterpret_cast<int32_t *>(ws + L.hl[t][3]);
  }
  a.gsz = reinterpret_cast<int32_t *>(ws + L.gsz);
  a.goff = reinterpret_cast<int32_t *>(ws + L.goff);
  a.gkey = reinterpret_cast<int32_t *>(ws + L.gkey);
  a.gval = reinterpret_cast<uint32_t *>(ws + L.gval);
  int32_t *tmp = reinterpret_cast<int32_t *>(ws + L.tmp);
  char *misc = ws + L.misc;
  a.tickets = reinterpret_cast<int32_t *>(misc);
  a.status = reinterpret_cast<int32_t *>(misc + 128);  // after 32 ticket counters
  a.hc = reinterpret_cast<int32_t *>(misc + 192);
  a.stats = stats;
  a.hubs = hubs && !local && g.wtype == SSSP_W_U32 && n <= HUB_NMAX && m > 0;
  a.hin = a.hubs ? reinterpret_cast<uint8_t *>(ws + L.hin) : nullptr;
  a.hout = a.hubs ? reinterpret_cast<uint8_t *>(ws + L.hout) : nullptr;
  a.hubm = a.hubs ? reinterpret_cast<int32_t *>(ws + L.hubm) : nullptr;
  uint32_t *kbits = out_row_ptr ? reinterpret_cast<uint32_t *>(ws + L.kbits) : nullptr;
  int32_t *kpre = out_row_ptr ? reinterpret_cast<int32_t *>(ws + L.kpre) : nullptr;
  *status_out = a.status;

  const int blocks = 2048;
  hipLaunchKernelGGL(k_tb_status, dim3(1), dim3(64), 0, st, a);
  if (validate && launch_validate(g, 1, 0, a.status, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tb_zero, dim3(blocks), dim3(256), 0, st, a);
  if (m > 0) {
    hipLaunchKernelGGL(k_tb_tilerow, dim3(blocks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_tb_tails, dim3(blocks), dim3(TL_BS), 0, st, a);
  }
  const int chunks = (int)(((long long)m + CCH - 1) / CCH);
  if (m > 0) {
    hipLaunchKernelGGL(k_csc_hist, dim3(L.tiles), dim3(C_BS), 0, st, a);
    if (launch_excl_scan(a.btot, L.nb, a.bstart, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
    hipLaunchKernelGGL(k_csc_scatter, dim3(L.tiles), dim3(C_BS), 0, st, a);
    hipLaunchKernelGGL(k_csc_count, dim3(chunks), dim3(C_BS), 0, st, a);
  }
  if (launch_excl_scan(a.ccnt, n, a.cb, tmp, st) != hipSuccess) return SSSP_ERR_HIP;
  // Side streams, unless st is being captured (then everything stays on st).
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return SSSP_ERR_HIP;
  std::unique_lock<std::mutex> side_lock;
  SideStreams *side = nullptr;
  if (cap == hipStreamCaptureStatusNone) {
    side_lock = std::unique_lock<std::mutex>(side_mutex());
    if (!(side = side_streams())) return SSSP_ERR_HIP;
  }
  // The u-side work estimate and the hub selection need only the CSR and
  // the column sizes: they run beside the CSC placement (which charges the
  // x-side work to the other half of `work`).
  hipStream_t ast = st;
  if (side) {
    if (hipEventRecord(side->ev[6], st) != hipSuccess ||
        hipStreamWaitEvent(side->s[1], side->ev[6], 0) != hipSuccess)
      return SSSP_ERR_HIP;
    ast = side->s[1];
  }
  hipLaunchKernelGGL(k_tb_work, dim3(blocks), dim3(256), 0, ast, a);
  if (a.hubs) {
    hipLaunchKernelGGL(k_hub_hist, dim3(grid_cus * 4), dim3(256), 0, ast, a);
    hipLaunchKernelGGL(k_hub_take, dim3(blocks), dim3(256), 0, ast, a);
  }
  if (side && hipEventRecord(side->ev[7], ast) != hipSuccess) return SSSP_ERR_HIP;
  if (m > 0) hipLaunchKernelGGL(k_csc_place, dim3(chunks), dim3(C_BS), 0, st, a);
  if (side && hipStreamWaitEvent(st, side->ev[7], 0) != hipSuccess) return SSSP_ERR_HIP;
  // the hubs' code rows read their CSC columns: after the placement, before
  // the cost order moves the entries
  if (a.hubs) hipLaunchKernelGGL(k_hub_tables, dim3(64, HUB_K), dim3(256), 0, st, a);
  // The cost order (lists of at most SORT_MAX entries) runs beside the
  // classification and the global tables (lists longer than HV_TCAP only):
  // they touch disjoint data, and the scans need both.
  hipStream_t ost = st;
  if (side) {
    if (hipEventRecord(side->ev[0], st) != hipSuccess ||
        hipStreamWaitEvent(side->s[0], side->ev[0], 0) != hipSuccess)
      return SSSP_ERR_HIP;
    ost = side->s[0];
  }
  static_assert(SORT_MAX <= HV_TCAP, "ordered lists never have a global table");
  hipLaunchKernelGGL(k_tb_sort_class, dim3(grid_cus), dim3(CLS_BS), 0, ost, a);
  hipLaunchKernelGGL(k_tb_sort_small, dim3(blocks), dim3(256), 0, ost, a);
  hipLaunchKernelGGL(k_tb_sort_mid, dim3(grid_cus * 8), dim3(ORD_BS), 0, ost, a);
  if (side && hipEventRecord(side->ev[1], ost) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tb_classify, dim3(grid_cus * 2), dim3(CLF_BS), 0, st, a);
  hipLaunchKernelGGL(k_tb_gclear, dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_tb_gtab, dim3(grid_cus, 16), dim3(256), 0, st, a);
  if (side && hipStreamWaitEvent(st, side->ev[1], 0) != hipSuccess) return SSSP_ERR_HIP;
  if (ev_start && hipEventRecord((hipEvent_t)ev_start, st) != hipSuccess) return SSSP_ERR_HIP;
  const hipError_t se = g.wtype == SSSP_W_U32
                            ? launch_scan_kernels<SSSP_W_U32>(a, grid_cus, st, side)
                            : launch_scan_kernels<SSSP_W_F32>(a, grid_cus, st, side);
  if (se != hipSuccess || hipGetLastError() != hipSuccess) return SSSP_ERR_HIP;
  if (ev_stop && hipEventRecord((hipEvent_t)ev_stop, st) != hipSuccess) return SSSP_ERR_HIP;
  hipLaunchKernelGGL(k_tb_count_pruned, dim3(512), dim3(256), 0, st, keep, m, stats, a.status);
  if (out_row_ptr) {
    const int ntiles = (int)(((long long)m + SCAN_TILE - 1) / SCAN_TILE);
    if (ntiles > 0)
      hipLaunchKernelGGL(k_keep_tiles, dim3(ntiles), dim3(KT_BS), 0, st, keep, m, kbits, kpre,
                         tmp);
    if (launch_scan_sums(tmp, ntiles, kpre + ((long long)m + 31) / 32, st) != hipSuccess)
      return SSSP_ERR_HIP;
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(256), 0, st, g.row_ptr, g.col,
                       static_cast<const uint32_t *>(g.w), keep, n, m, kbits, kpre, tmp,
                       out_row_ptr, out_col, static_cast<uint32_t *>(out_w), edge_map,
                       a.status);
  }
  hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st, a.status, stats);
  return hipGetLastError() == hipSuccess ? SSSP_OK : SSSP_ERR_HIP;
}

}  // namespace sssp_impl
