// internal.hpp -- device helpers and launch descriptors shared by the
// library's kernels (gfx950, wave64).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sssp.h"

namespace sssp_impl {

constexpr int WAVE = 64;
constexpr uint32_t NONE_EDGE = 0xFFFFFFFFu;
constexpr unsigned long long LABEL_INF = ~0ull;
constexpr unsigned long long DELTA_INF = ~0ull;
constexpr unsigned long long DELTA_AUTO = 0ull;  // bucket width set on the device
constexpr int ABW_STRIDE = 32;                   // active-unit bitmap word stride
constexpr int ABW_UNITS = 8;                     // units per active-unit bitmap word

// How a partition settles its vertices inside a batch (k_solve's MODE).
enum SolveMode {
  SOLVE_BUCKETS = 0,   // delta buckets, cross-partition labels updated at once
  SOLVE_BUFFERED = 1,  // delta buckets, cross-partition updates buffered per head
  SOLVE_HEAP = 2,      // one vertex at a time from an LDS binary heap
  SOLVE_IDLE_PRUNE = 3 // delta buckets; idle workgroups prune (LOCAL Trishla)
};
constexpr int PRUNE_CHUNK = 64;  // vertices per idle-pruning ticket

// ------------------------------------------------------------ atomics
// Every datum that several workgroups write or read while a kernel runs is
// accessed with agent-scope atomics: the eight XCDs have private L2 caches,
// so plain loads could observe stale lines.
template <typename T>
__device__ __forceinline__ T ld_acq(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_rlx(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_rlx(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_rel(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T amin(T *p, T v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T amax(T *p, T v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T aadd(T *p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T aor(T *p, T v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T aand_acq(T *p, T v) {
  return __hip_atomic_fetch_and(p, v, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_status(int32_t *st, int32_t code) {
  int32_t expect = 0;
  __hip_atomic_compare_exchange_strong(st, &expect, code, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ uniform values
// Values read from LDS are uniform across the workgroup but the compiler
// cannot prove it; moving them to scalar registers frees vector registers.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ unsigned long long uni64(unsigned long long x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
template <typename T>
__device__ __forceinline__ T *uni_ptr(T *p) {
  return reinterpret_cast<T *>(uni64(reinterpret_cast<unsigned long long>(p)));
}

// Hides a uniform pointer's value from the optimiser (no instruction is
// emitted), so addresses derived from it inside a persistent loop are
// recomputed each iteration instead of being hoisted and kept live.
template <typename T>
__device__ __forceinline__ T *opaque(T *p) {
  unsigned long long x = reinterpret_cast<unsigned long long>(p);
  asm volatile("" : "+s"(x));
  return reinterpret_cast<T *>(x);
}

// Same for a per-lane value (e.g. the thread index) inside a persistent loop.
__device__ __forceinline__ int opaque_v(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// ------------------------------------------------------------ wave / block
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_min(T x) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o, WAVE);
    x = y < x ? y : x;
  }
  return x;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan of one int per thread over the block.  `ws` holds
// BS/64 + 1 ints of LDS.  Returns the exclusive prefix; *total = block sum.
template <int BS>
__device__ __forceinline__ int block_excl_scan(int x, int *ws, int *total) {
  constexpr int NW = BS / WAVE;
  const int wid = threadIdx.x / WAVE;
  int incl = wave_incl_scan(x);
  if (lane_id() == WAVE - 1) ws[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      int t = ws[i];
      ws[i] = acc;
      acc += t;
    }
    ws[NW] = acc;
  }
  __syncthreads();
  int r = ws[wid] + incl - x;
  *total = ws[NW];
  __syncthreads();
  return r;
}

// Exclusive scan of one int per thread over the block with a single
// barrier: every thread adds up the totals of the waves before its own.
// ws (BS/64 ints) must not be written again before another barrier.
template <int BS>
__device__ __forceinline__ int block_excl_scan1(int x, int *ws, int *total) {
  constexpr int NW = BS / WAVE;
  const int wid = threadIdx.x / WAVE;
  const int incl = wave_incl_scan(x);
  if (lane_id() == WAVE - 1) ws[wid] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NW; k++) {
    const int t = ws[k];
    before += k < wid ? t : 0;
    all += t;
  }
  *total = all;
  return before + incl - x;
}

// ------------------------------------------------------------ solve descriptors
// One independent single-source problem of a (possibly batched) solve.
struct SolveDesc {
  const int32_t *row_ptr;
  const int32_t *col;
  const uint32_t *w;           // raw 32-bit weights (uint32 or float32 bits)
  unsigned long long *label;   // n packed labels: dist bits << 32 | edge id
  uint32_t *dirty;             // ceil(n/32) words: the partitions' inboxes
  void *dist;                  // outputs, already offset for this solve
  int32_t *pred;
  int32_t *pred_edge;
  unsigned long long delta;    // bucket width in dist units, DELTA_INF = none
  int32_t n, m, source;
  int32_t nparts, bsize;       // P and the 1D block size ceil(n/P)
  int32_t unit0;               // first scheduling unit (partition) index
  int32_t nwords;              // ceil(n/32)
  float auto_factor;           // DELTA_AUTO: width = factor * mean sampled cost
};

// Device-wide control block living in the workspace.  The pending-work
// counter has a 128-byte line to itself: its atomics do not slow the loads
// of the flags that every workgroup polls.
struct Ctrl {
  long long work;   // pending work: inbox bits + claimed vertices (+ raises)
  uint32_t pad_w[30];
  uint32_t done;    // set once the solve has finished or aborted
  int32_t status;   // first device-detected error
  uint32_t nunits;
  uint32_t ovf;     // a relaxation candidate did not fit the distance type
  unsigned long long window;  // bounded lag in dist units (DELTA_INF = none)
  int32_t prune_next;         // SOLVE_IDLE_PRUNE: next prune ticket
  uint32_t pad[25];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl layout");

// Kernel arguments of the persistent solve.
struct SolveArgs {
  const SolveDesc *desc;       // num_solves descriptors
  int32_t *unit_solve;         // unit -> solve index
  unsigned long long *unit_min;  // per unit: least pending distance (lower bound)
  uint32_t *abits;             // active-unit bitmap, one 8-unit word per
                               // 128-byte line (ABW_STRIDE words apart)
  Ctrl *ctrl;
  sssp_stats *stats;
  int32_t nunits, nabw;        // units, words of abits
  int32_t max_rounds;
  int32_t num_solves;
  unsigned long long window;      // bounded lag (copied to Ctrl::window)
  unsigned long long time_limit;  // wall-clock ticks
  int32_t auto_lag;               // > 0: single solve with DELTA_AUTO, window = lag * width
  int32_t prune_tasks;            // SOLVE_IDLE_PRUNE: vertex chunks idle workgroups prune
  uint32_t *keepbits;             //   one bit per arc of solve 0, 1 = kept
  uint8_t *keep_out;              //   optional uint8[m] copy of the bits after the solve
  int32_t desc_m0;                //   arcs of solve 0
  int32_t pad;
};

// Descriptors travel to the device inside kernel arguments (below 4 KiB).
struct DescChunk {
  int32_t first, count;
  SolveDesc d[32];
};

__device__ __forceinline__ void stat_add(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace sssp_impl
