/*
 * sssp.h -- C ABI of the MI355X (gfx950) partitioned single-source
 * shortest-path library: Trishla pruning, asynchronous partitioned solve,
 * batched solve and the weight gradient of the distances.
 *
 * Problem (Sec. I): a directed graph G(V,E) in CSR form, a source s and a
 * nonnegative cost on every arc; the library computes d(v), the least total
 * cost of an s->v path, and a shortest-path tree.
 *
 * Common conventions
 *   - Every array argument named "device" is memory on the current HIP
 *     device; "host" arrays are read during the call only.
 *   - The caller owns and allocates every buffer, including the workspace.
 *     The library never allocates or frees device memory during a call.
 *   - Workspace protocol: call with ws == NULL to have the required size in
 *     bytes written to *ws_bytes (returns SSSP_OK, enqueues nothing); then
 *     call again with ws pointing to at least that many bytes (256-byte
 *     aligned) and *ws_bytes holding its size.
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream) and the call returns without waiting, unless SSSP_F_SYNC is
 *     set.  Calls without SSSP_F_SYNC perform no allocation, no host<->device
 *     copy and no synchronisation, so they may be captured into a HIP graph.
 *   - Errors found on the host are returned before anything is enqueued.
 *     Errors found on the device are written to stats->status (when stats is
 *     non-NULL) and, with SSSP_F_SYNC, returned.
 *   - Distances: uint32 weights give uint32 distances with 0xFFFFFFFF for
 *     unreachable vertices; float32 weights give float32 distances with +inf
 *     for unreachable vertices, accumulated as fl32(d(u) + w) (round to
 *     nearest even) along the path.
 *   - Predecessors: pred_edge[v] is the smallest edge id e = (u,v) with
 *     d(u) + w_e == d(v) (a tight arc), pred[v] its tail u; both are -1 for
 *     the source and for unreachable vertices.  Edge ids are positions in
 *     the `col` array of the CSR passed to that call.
 */
#ifndef SSSP_H
#define SSSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
enum {
  SSSP_OK = 0,
  SSSP_ERR_ARG = -1,          /* null pointer, bad size, bad option        */
  SSSP_ERR_SOURCE = -2,       /* source outside [0, n)                     */
  SSSP_ERR_CSR = -3,          /* row_ptr not monotone / != m, col out of range */
  SSSP_ERR_UNSORTED = -4,     /* sssp_prune: a row is not sorted by column */
  SSSP_ERR_WEIGHT = -5,       /* fp32 weight negative, -0.0, NaN or inf    */
  SSSP_ERR_ZERO_WEIGHT = -6,  /* sssp_backward: a weight equal to zero     */
  SSSP_ERR_OVERFLOW = -7,     /* a final distance does not fit: an integer
                                 distance reaches 2^32 - 1, or a reachable
                                 vertex's fp32 distance is +inf.  A longer
                                 path whose sum does not fit is no error    */
  SSSP_ERR_TIMEOUT = -8,      /* max_rounds or the time limit was reached  */
  SSSP_ERR_WORKSPACE = -9,    /* workspace missing, too small or misaligned */
  SSSP_ERR_HIP = -10,         /* a HIP runtime call failed                 */
  SSSP_ERR_CAPTURE = -11,     /* SSSP_F_SYNC requested on a capturing stream */
  SSSP_ERR_CYCLE = -12,       /* sssp_backward: predecessors form a cycle  */
  SSSP_ERR_TOO_LARGE = -13    /* sssp_solve_noalloc: the solve needs more than
                                 SSSP_NOALLOC_SCRATCH_BYTES of workspace   */
};

/* Human-readable name of an error code (static string, never NULL). */
const char *sssp_strerror(int code);

/* ------------------------------------------------------------ the graph */
enum { SSSP_W_U32 = 0, SSSP_W_F32 = 1 };

/* Largest graphs accepted (else SSSP_ERR_ARG): 32-bit vertex and arc
 * indices, with room for twice the vertex count and for grid-stride steps
 * without integer overflow in the kernels. */
#define SSSP_N_MAX ((1 << 30) - (1 << 24))
#define SSSP_M_MAX (0x7FFFFFFF - (1 << 24) + 1)

typedef struct {
  int32_t n;              /* number of vertices, 1 <= n <= SSSP_N_MAX      */
  int32_t m;              /* number of arcs, 0 <= m <= SSSP_M_MAX          */
  const int32_t *row_ptr; /* device int32[n+1]: row_ptr[0] = 0, nondecreasing,
                             row_ptr[n] = m; arcs of u are row_ptr[u]..row_ptr[u+1]-1 */
  const int32_t *col;     /* device int32[m]: head of every arc, in [0, n)  */
  const void *w;          /* device uint32[m] or float32[m]: arc costs >= 0 */
  int32_t wtype;          /* SSSP_W_U32 or SSSP_W_F32                      */
  int32_t reserved;       /* must be 0                                     */
} sssp_csr;

/* --------------------------------------------------------------- options */
enum {
  SSSP_F_VALIDATE = 1u << 0,     /* check CSR and weights on the device first */
  SSSP_F_SYNC = 1u << 1,         /* wait for completion, return device status  */
  SSSP_F_PRUNE_LOCAL = 1u << 2,  /* sssp_prune: LOCAL scope (witness in u's partition) */
  SSSP_F_NO_AUTOTUNE = 1u << 3,  /* never consult the autotune cache           */
  /* sssp_solve / sssp_solve_batch: buffer cross-partition label updates.  A
     candidate label for a head in another partition is kept in a per-batch
     LDS table that holds the least candidate per head, and each distinct
     head is updated once, at the end of each settle round, when the table
     is full (the overflow goes straight to HBM) and at the end of the batch
     (the message buffering the paper names as future work, Sec. V, with
     min-combining).  Results are the same; only the number of global
     atomics and the timing change. */
  SSSP_F_BUFFER_CROSS = 1u << 4,
  /* sssp_solve / sssp_solve_batch: the paper's local rule taken literally
     (Alg. 3): a partition settles its vertices one at a time from a binary
     heap in LDS, least tentative distance first, pushing every improved
     head of its own partition and sending the others to their owners'
     inboxes, until its heap is empty (or 256 pops; the rest goes back to
     the inbox).  delta plays no part in a batch (the lag window still
     bounds which partitions may run).  Results are the same.  Not together
     with SSSP_F_BUFFER_CROSS (SSSP_ERR_ARG). */
  SSSP_F_LOCAL_HEAP = 1u << 5,
  /* sssp_solve only: idle-time pruning (Sec. III-B: processes that receive
     no message prune their subgraph meanwhile, and the solve skips what
     they delete; Sec. II: pruning overlapped with the SSSP computation).
     A workgroup that finds no partition to settle runs Trishla with LOCAL
     scope (the middle vertex in the tail's own partition) over a chunk of
     64 vertices and marks the arcs it deletes; the solve no longer relaxes
     them.  Which arcs are deleted depends on timing (a row of more than
     1024 arcs or more than 65536 two-arc paths is skipped, and the solve
     ends when no work is pending, pruned or not), but every deleted arc is
     in the LOCAL deletion set, so distances and predecessors are the same.
     opts->keep_out, if set, receives the keep flags; stats->edges_pruned and
     stats->wedges count deleted arcs and two-arc paths examined.  Not
     together with the two modes above (SSSP_ERR_ARG). */
  SSSP_F_IDLE_PRUNE = 1u << 6,
  /* sssp_prune: skip the hub pass (the arcs are tested through the
     32 vertices with the most two-arc paths first, with integer
     costs, GLOBAL scope and n <= 2^23); the result is the same, only the
     time changes.  For comparisons. */
  SSSP_F_PRUNE_NO_HUBS = 1u << 7
};

typedef struct {
  double delta;            /* bucket width (distance units); < 0 or +inf =
                              one unbounded bucket; 0 = auto: the autotune
                              cache entry for this graph's signature, else
                              computed on the device as a multiple of the
                              mean of sampled arc costs (0.5x when the
                              average degree is >= 8, 16x below)          */
  int32_t num_partitions;  /* P, 1D blocks of ceil(n/P) vertices; 0 = auto
                              (cache, else blocks of 4096 vertices when the
                              average degree is >= 8 and 65536 below);
                              raised so that a block has at most 65536 vertices */
  int32_t wg_size;         /* threads per workgroup: 256, 512 or 1024; 0 = auto
                              (cache, else 512 when the average degree is
                              >= 8 and 256 below)                          */
  int32_t num_workgroups;  /* persistent grid size; 0 = auto (cache, else one
                              workgroup per CU when the average degree is
                              >= 8 and two below); capped by residency     */
  int32_t max_rounds;      /* > 0: stop after this many frontier batches per
                              workgroup and report SSSP_ERR_TIMEOUT; the
                              labels are then valid upper bounds           */
  uint32_t flags;          /* SSSP_F_* */
  int32_t lag;             /* sssp_solve: a partition may expand its lowest
                              bucket only while its pending minimum is within
                              lag * delta of the least pending distance of the
                              whole graph; 0 = auto (the autotune cache,
                              else 1), < 0 = unbounded (fully
                              asynchronous partitions).  Batched solves are
                              always unbounded.  Results never depend on it. */
  void *event_start;       /* optional hipEvent_t recorded right before the
                              main kernel of the call (NULL = none)        */
  void *event_stop;        /* optional hipEvent_t recorded right after it  */
  void *keep_out;          /* SSSP_F_IDLE_PRUNE: optional device uint8[m]
                              receiving 1 for every arc kept and 0 for every
                              arc deleted during the solve (NULL = none)   */
} sssp_opts;

/* Fill *o with the defaults (everything automatic). */
void sssp_opts_init(sssp_opts *o);

/* --------------------------------------------------------------- stats */
/* Device-resident counters, optional (NULL = not collected).  The library
 * zeroes the struct at the start of each call. */
typedef struct {
  int32_t status;            /* SSSP_OK or a device-detected SSSP_ERR_*    */
  int32_t num_partitions;    /* P actually used                            */
  uint64_t delta_bits;       /* bucket width used (integer, or fp32 bits)  */
  uint64_t edges_relaxed;    /* arcs examined by the solve                 */
  uint64_t label_updates;    /* atomic min operations that lowered d(v)   */
  uint64_t cross_updates;    /* of those, arcs into another partition     */
  uint64_t vertices_expanded;/* frontier vertices processed (with repeats) */
  uint64_t batches;          /* frontier batches (bucket rounds)          */
  uint64_t edges_pruned;     /* sssp_prune: arcs deleted                   */
  uint64_t wedges;           /* sssp_prune: list entries examined by the
                                scans (candidate two-arc paths)           */
  uint64_t hub_pruned;       /* sssp_prune: arcs deleted by the hub pass
                                (included in edges_pruned)                */
  uint64_t reserved[5];
} sssp_stats;

/* --------------------------------------------------------------- prune */
/*
 * Trishla (Sec. III-B, Alg. 1): delete every arc e = (u,x,W) for which some
 * middle vertex y, y != u and y != x, has arcs (u,y,w1) and (y,x,w2) with
 * w1 + w2 < W (strict; integer sums in 64 bits, fp32 sums compared exactly).
 * All arcs are tested against the input graph at once.  Scope GLOBAL
 * (default) allows any y; SSSP_F_PRUNE_LOCAL requires y to lie in u's 1D
 * partition (Sec. III-A).  With integer costs, deleting such arcs never
 * changes a distance nor the predecessor rule's choice (a deleted arc is
 * never tight).  With fp32 costs the same holds for exact sums; the solve,
 * however, rounds every fp32 sum, so on a pruned fp32 graph a rounded
 * distance may come out a few ulps different (e.g. d(u) = 2^24 + 2,
 * w1 = 1, w2 = 1.5, W = 2.9: the arc of cost W is deleted because
 * 2.5 < 2.9, but fl(fl(d(u) + 1) + 1.5) = 2^24 + 6 > fl(d(u) + 2.9) =
 * 2^24 + 4).
 *
 * Requires every row sorted by column (nondecreasing).
 *   keep            device uint8[m]: 1 = kept, 0 = deleted              (out)
 *   out_row_ptr     device int32[n+1] or NULL: CSR of the kept arcs    (out)
 *   out_col, out_w  device int32[m], device uint32/float32[m], or NULL (out)
 *   edge_map        device int32[m] or NULL: original id of kept arc i (out)
 * Kept arcs stay in their original order; the kept count is
 * out_row_ptr[n].  The out_* arrays and edge_map must be all NULL or all set.
 * The work is ordered on `stream` as one unit.  Part of it runs on three
 * library-owned streams of the current device, forked from `stream` and
 * joined back with events.  Those streams and events are created on the
 * first call and kept until the process ends.  Under stream capture
 * everything stays on `stream`.
 */
int sssp_prune(const sssp_csr *g, const sssp_opts *o, uint8_t *keep,
               int32_t *out_row_ptr, int32_t *out_col, void *out_w,
               int32_t *edge_map, sssp_stats *stats, void *ws,
               size_t *ws_bytes, void *stream);

/* --------------------------------------------------------------- solve */
/*
 * Single-source shortest paths (Sec. III-C, Alg. 2 and 3) over 1D vertex
 * partitions (Sec. III-A).  Each partition settles its vertices in order of
 * delta-wide distance buckets (lowest non-empty bucket first); arcs into
 * other partitions are relaxed immediately with a 64-bit atomic minimum on
 * the packed (distance, edge id) label of the head and mark the head in its
 * owner's inbox -- the asynchronous Bellman-Ford exchange between
 * partitions.  A device-wide count of pending work replaces the paper's
 * termination detection (Sec. III-D): the solve ends when it reaches zero.
 * The result does not depend on delta, P, the grid or the schedule.  A
 * relaxation candidate that does not fit the distance type is skipped;
 * after the solve, SSSP_ERR_OVERFLOW is reported if and only if some final
 * distance does not fit (an arc from a reached vertex into a vertex left
 * unreached), which is again independent of the schedule.
 *   dist        device uint32[n] or float32[n] (per g->wtype)          (out)
 *   pred        device int32[n] or NULL                                (out)
 *   pred_edge   device int32[n] or NULL                                (out)
 */
int sssp_solve(const sssp_csr *g, int32_t source, const sssp_opts *o,
               void *dist, int32_t *pred, int32_t *pred_edge,
               sssp_stats *stats, void *ws, size_t *ws_bytes, void *stream);

/* ---------------------------------------------------------- batched solve */
/*
 * A project layer over sssp_solve (not a step of the paper): many
 * independent single-source problems in one persistent launch.  Sec. IV runs
 * the pruning once per graph and the two remaining phases once per source;
 * this entry point runs those per-source phases of many (graph, source)
 * pairs together, each pair's partitions being scheduling units of one
 * shared unit space.  Solve i runs on graph
 * solve_graph[i] (an index into `graphs`) from solve_source[i] and writes
 * its n_i outputs at element offset out_offset[i] of dist / pred /
 * pred_edge.  Each solve's result equals sssp_solve on the same input.
 *   graphs        host sssp_csr[num_graphs] (device pointers inside)
 *   solve_graph, solve_source   host int32[num_solves]
 *   out_offset    host int64[num_solves]
 *   dist          device uint32/float32[total], pred / pred_edge device
 *                 int32[total] or NULL
 * All graphs must share one wtype.  The task table is passed to the device
 * inside kernel arguments, so a captured call replays without the host
 * arrays.  opts->num_partitions applies per graph (0 = auto per graph).
 */
int sssp_solve_batch(int32_t num_graphs, const sssp_csr *graphs,
                     int32_t num_solves, const int32_t *solve_graph,
                     const int32_t *solve_source, const int64_t *out_offset,
                     const sssp_opts *o, void *dist, int32_t *pred,
                     int32_t *pred_edge, sssp_stats *stats, void *ws,
                     size_t *ws_bytes, void *stream);

/* ------------------------------------------------------------ backward */
/*
 * Gradient of L = sum_v grad_dist[v] * d(v) with respect to every arc cost,
 * for fp32 graphs (not in the paper).  d(t) is the sum of the costs on the
 * tree path s -> t, so grad_w[e] = sum of grad_dist[t] over the vertices t
 * whose tree path uses e: for e = pred_edge[v] it is the total of
 * grad_dist over the subtree under v, and 0 for every other arc.  Subtree
 * totals are accumulated in reverse distance order (children before their
 * parent) in float64 and rounded once to float32.
 * Requires every weight > 0 (else SSSP_ERR_ZERO_WEIGHT, checked with
 * SSSP_F_VALIDATE); a predecessor cycle is reported as SSSP_ERR_CYCLE.
 *   dist, pred_edge   device float32[n], int32[n]: the output of sssp_solve
 *   grad_dist         device float32[n] (entries of unreachable v ignored)
 *   grad_w            device float32[m]                                (out)
 */
int sssp_backward(const sssp_csr *g, int32_t source, const float *dist,
                  const int32_t *pred_edge, const float *grad_dist,
                  float *grad_w, const sssp_opts *o, sssp_stats *stats,
                  void *ws, size_t *ws_bytes, void *stream);

/* ------------------------------------------------------------ autotune */
/*
 * Time candidate (delta, num_partitions, wg_size, num_workgroups, lag) settings for
 * sssp_solve on this graph and source and write the fastest into *best
 * (synchronous; not for capture).  *best is in/out: fields the caller sets
 * to nonzero values (delta, num_partitions, wg_size, num_workgroups, lag)
 * are kept fixed, the others are searched (delta over multiples of the mean
 * arc cost sampled from the device, and one unbounded bucket).  Results
 * are cached in the process, keyed by the device and a signature of the
 * graph (weight type, ceil(log2 n), floor(log2) of the average degree), and
 * sssp_solve with automatic options consults the cache.  If cache_path is
 * non-NULL the cache is loaded from and saved to that JSON file.  The
 * bucket-width trade-off it searches is the one the paper's discussion of
 * delta-stepping describes (wider buckets: more parallel work, more
 * re-relaxation).
 *   dist_scratch  device buffer of 4*n bytes used as the dist output
 */
int sssp_autotune(const sssp_csr *g, int32_t source, void *dist_scratch,
                  sssp_opts *best, const char *cache_path, void *ws,
                  size_t *ws_bytes, void *stream);

/*
 * The same for one sssp_solve_batch call: times settings of the whole
 * batched launch (delta: each graph's automatic width or one shared
 * multiple of the mean cost of graphs[0]; num_partitions: each graph's
 * default or one shared count; wg_size; num_workgroups) and writes the
 * fastest into *best (in/out as above; lag does not apply to batches).  The
 * result is cached under a signature of the batch (weight type, number of
 * graphs and solves, ceil(log2) of the total vertex count, floor(log2) of
 * the average degree); sssp_solve_batch with automatic options consults only
 * such batch entries.  Arguments as in sssp_solve_batch, plus:
 *   dist_scratch  device buffer holding the batch's dist output
 *                 (4 * max(out_offset[s] + n of solve s) bytes)
 * Workspace protocol as everywhere (ws == NULL queries the largest
 * requirement over the candidates).  Synchronous; not for capture.
 */
int sssp_autotune_batch(int32_t num_graphs, const sssp_csr *graphs, int32_t num_solves,
                        const int32_t *solve_graph, const int32_t *solve_source,
                        const int64_t *out_offset, void *dist_scratch, sssp_opts *best,
                        const char *cache_path, void *ws, size_t *ws_bytes, void *stream);

/* ----------------------------------------------------- solve, no allocation */
/*
 * For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * sssp_solve with the same arguments and results, minus the workspace.  The
 * workspace is a fixed array of SSSP_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held from module load until the process ends.  A
 * graph whose solve needs more (as sssp_solve's ws == NULL query reports;
 * about 8 million vertices) is rejected with SSSP_ERR_TOO_LARGE before
 * anything is enqueued.  The call allocates nothing; its first call on a
 * device looks up that device's array address (hipGetSymbolAddress).  All
 * calls on one GPU share its array: calls that overlap on one GPU (on
 * different streams or host threads) race and must be ordered by the
 * caller; calls in one stream are ordered already.
 */
#define SSSP_NOALLOC_SCRATCH_BYTES (64u << 20)
int sssp_solve_noalloc(const sssp_csr *g, int32_t source, const sssp_opts *o,
                       void *dist, int32_t *pred, int32_t *pred_edge,
                       sssp_stats *stats, void *stream);

/* Library version string. */
const char *sssp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SSSP_H */
