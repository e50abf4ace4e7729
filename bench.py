"""Benchmark of the SP-Async hot path on one MI355X.

Default workload (the headline line): R-MAT scale 20 (edge factor 16,
a/b/c/d = .57/.19/.19/.05, duplicates and self-loops removed), uint32 costs
uniform on {1..255}; one step = Trishla pruning of the whole graph, then a
single-source solve of the pruned graph from a random non-isolated source
with 256 partitions.  GTEPS = arcs of the input graph whose tail is reached,
per second of step time.  Inputs are resident in HBM before timing starts.

Extra measurements on the same GPU (reported under "extra"): the road-like
4096x4096 grid solve, the batched solve (64 R-MAT graphs of scales 12..18,
4 sources each, one captured launch) against 256 single-source calls, the
differentiable R-MAT scale-22 forward + backward, and an ablation of the
local rule (bucket width 1 = exact local distance order, one unbounded
bucket = asynchronous Bellman-Ford, automatic width) on the headline graph.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only NAME ...]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS and % HBM roofline, single-source vs batched; backward ms at 1e-4 tol"
HBM_PEAK_GBS = 8000.0


# ------------------------------------------------------------------ HIP events
class HipEvents:
    """Raw hipEvent_t pairs (recorded by the library around its main kernel,
    on the stream that kernel runs on)."""

    def __init__(self):
        self.h = ctypes.CDLL("libamdhip64.so")
        self.h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.h.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.h.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def pair(self):
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        assert self.h.hipEventCreate(ctypes.byref(a)) == 0
        assert self.h.hipEventCreate(ctypes.byref(b)) == 0
        return a.value, b.value

    def ms(self, pair):
        self.h.hipEventSynchronize(ctypes.c_void_p(pair[1]))
        out = ctypes.c_float()
        assert self.h.hipEventElapsedTime(ctypes.byref(out), ctypes.c_void_p(pair[0]),
                                          ctypes.c_void_p(pair[1])) == 0
        return float(out.value)


def m_reached(g, source):
    from paper_2103_12012_amd import gen

    mask = gen.reachable_mask(g, source)
    return int(g.out_degree()[mask].sum()), int(mask.sum())


KERNEL_SOURCES = {  # files each kernel is compiled from (for the counter-staleness check)
    "k_solve": ("internal.hpp", "solve.hip"),
    "k_tb_light": ("internal.hpp", "prune.hip"),
    # heavy owners by list length: <= 512, <= 1024, <= 2048 entries, and longer
    "k_tb_heavy_t0": ("internal.hpp", "prune.hip"),
    "k_tb_heavy_t1": ("internal.hpp", "prune.hip"),
    "k_tb_heavy_t2": ("internal.hpp", "prune.hip"),
    "k_tb_heavy_big": ("internal.hpp", "prune.hip"),
    # every kernel of sssp_backward (clear, parents, marks, counts, leaves, chains, check)
    "k_bwd": ("internal.hpp", "backward.hip"),
}
TRISHLA_SCAN = ("k_tb_light", "k_tb_heavy_t0", "k_tb_heavy_t1", "k_tb_heavy_t2", "k_tb_heavy_big")


def kernel_source_hash(kernel):
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2103_12012_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary profiles/pmc_<kernel>_<workload>.txt: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch, one --pmc run each), each scaled by the factor the same
    counter gives for a plain device copy of known size.  None when there is
    no summary or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#", "-")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("source_sha256") != kernel_source_hash(kernel):
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 * float(kv["copy_fetch_factor"])
        write = float(kv["write_kib_per_dispatch"]) * 1024 * float(kv["copy_write_factor"])
    except (KeyError, ValueError):
        return None
    return int(fetch + write)


def roofline(name, bytes_alg, ms, bound="hbm", workload=None, parts=None):
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    traffic = None
    if workload:
        ts = [counter_traffic(k, workload) for k in (parts or (name,))]
        traffic = None if any(t is None for t in ts) else sum(ts)
    return {"bound": bound, "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": name,
            "avg_launch_ms": round(ms, 4), "algorithmic_bytes": int(bytes_alg)}


# ------------------------------------------------------------------ headline
def bench_rmat20(steps, warmup, cpu_leg=True, tune=True):
    import torch

    from paper_2103_12012_amd import gen, sssp

    t0 = time.time()
    g = gen.rmat(20, 20)
    s = int(gen.random_sources(g, 1, 20)[0])
    mcc, ncc = m_reached(g, s)
    print(f"[bench] rmat20 n={g.n} m={g.m} source={s} m_cc={mcc} ({time.time()-t0:.1f}s gen)",
          file=sys.stderr, flush=True)
    rp, c, w = sssp.to_device(g, "cuda")
    P = 256
    ev = HipEvents()
    # buffers allocated once; one step = prune (with compaction) + solve
    L = sssp.lib()
    gcsr = sssp._csr(rp, c, w)
    popt = sssp.make_opts(num_partitions=P, validate=False)
    dev = "cuda"
    out_rp = torch.empty(g.n + 1, dtype=torch.int32, device=dev)
    out_c = torch.empty(g.m, dtype=torch.int32, device=dev)
    out_w = torch.empty(g.m, dtype=torch.int32, device=dev)
    emap = torch.empty(g.m, dtype=torch.int32, device=dev)
    keep = torch.empty(g.m, dtype=torch.uint8, device=dev)
    outs = [sssp._ptr(t) for t in (out_rp, out_c, out_w, emap)]
    nb = ctypes.c_size_t(0)
    assert L.sssp_prune(ctypes.byref(gcsr), ctypes.byref(popt), None, *outs, None, None,
                        ctypes.byref(nb), None) == 0
    pws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    # validate the input once, outside the timed loop
    sssp.prune(rp, c, w, num_partitions=P, validate=True)
    torch.cuda.synchronize()
    kept_m = None

    def prune_step(events=None):
        o = sssp.Opts.from_buffer_copy(popt)
        if events:
            o.event_start, o.event_stop = events
        n2 = ctypes.c_size_t(pws.numel())
        rc = L.sssp_prune(ctypes.byref(gcsr), ctypes.byref(o), sssp._ptr(keep), *outs, None,
                          sssp._ptr(pws), ctypes.byref(n2), sssp._stream())
        assert rc == 0, rc

    prune_step()
    torch.cuda.synchronize()
    kept_m = int(out_rp[-1].item())
    # one prune with counters: arcs deleted and list entries examined
    pst = sssp.StatsBuffer.new(dev)
    o = sssp.Opts.from_buffer_copy(popt)
    n2 = ctypes.c_size_t(pws.numel())
    assert L.sssp_prune(ctypes.byref(gcsr), ctypes.byref(o), sssp._ptr(keep), *outs,
                        sssp._ptr(pst.t), sssp._ptr(pws), ctypes.byref(n2), sssp._stream()) == 0
    torch.cuda.synchronize()
    prune_stats = pst.read()
    pg = (out_rp, out_c[:kept_m], out_w[:kept_m])
    # autotune the solve of the pruned graph (P fixed at 256; timed from this
    # source and four others, scored by the median) and compare with the
    # library defaults on this source; the step itself runs with the
    # defaults (the configuration fixes P only)
    ev0 = HipEvents()

    def solve_ms(sv, reps=10):
        sv(s)
        ts = []
        for _ in range(reps):
            e = ev0.pair()
            sv(s, events=e)
            ts.append(ev0.ms(e))
        return float(np.median(ts))

    if tune:
        tuned = sssp.autotune(*pg, s, num_partitions=P)
        sv_def = sssp.Solver(*pg, num_partitions=P, validate=False, no_autotune=True)
        sv_tun = sssp.Solver(*pg, num_partitions=P, validate=False)
        # interleaved, so that drift of the device's clocks hits both alike
        dts, tts = [], []
        for _ in range(10):
            dts.append(solve_ms(sv_def, 1))
            tts.append(solve_ms(sv_tun, 1))
        default_ms, tuned_ms = float(np.median(dts)), float(np.median(tts))
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        same = (tuned["delta"] == 0 and tuned["wg_size"] in (0, 512) and tuned["lag"] == 0
                and tuned["num_workgroups"] in (0, cus))  # one 512-thread workgroup per CU
        autotune_res = {"tuned_options": tuned, "solve_ms_default_options": round(default_ms, 4),
                        "solve_ms_tuned_options": round(tuned_ms, 4),
                        "tuned_equals_defaults": bool(same),
                        "note": "medians of 10 interleaved solves of the pruned graph from the "
                                "headline source"}
    else:
        autotune_res = {"skipped": True}
    solver = sssp.Solver(*pg, num_partitions=P, validate=False, stats=True, no_autotune=True)
    for _ in range(warmup):
        prune_step()
        solver(s)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        prune_step()
        solver(s)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = t_total / steps * 1e3
    # per-kernel device times: HIP events recorded by the library around its
    # main kernel on the launch stream; whole-step times with stream events.
    # The last-level cache (MALL) is flushed before each trial.
    flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    pr, so, whole = [], [], []
    for _ in range(max(10, steps)):
        flush.fill_(1)
        e1 = ev.pair()
        e2 = ev.pair()
        t0e = torch.cuda.Event(enable_timing=True)
        t1e = torch.cuda.Event(enable_timing=True)
        t0e.record()
        prune_step(e1)
        solver(s, events=e2)
        t1e.record()
        torch.cuda.synchronize()
        pr.append(ev.ms(e1))
        so.append(ev.ms(e2))
        whole.append(t0e.elapsed_time(t1e))
    del flush
    st = solver.stats.read()
    dist = solver.dist.cpu().numpy().view(np.uint32)
    reached = int((dist != 0xFFFFFFFF).sum())
    assert reached == ncc, (reached, ncc)
    prune_ms, solve_ms = float(np.mean(pr)), float(np.mean(so))
    # algorithmic bytes of the solve (per launch): init 8 B + epilogue 16 B per
    # vertex, 16 B per reached vertex (row bounds + own label), 16 B per arc
    # out of a reached vertex (col + cost + head label) in the pruned graph
    mr_pruned = int(np.diff(out_rp.cpu().numpy().astype(np.int64))[dist != 0xFFFFFFFF].sum())
    b_solve = 24 * g.n + 16 * reached + 16 * mr_pruned
    # Trishla: read CSR (8 B / arc + row pointers), keep flags, compacted CSR
    b_prune = 4 * (g.n + 1) + 8 * g.m + g.m + 4 * (g.n + 1) + 12 * kept_m
    rp_prune = roofline("trishla_scan", b_prune, prune_ms, workload="rmat20", parts=TRISHLA_SCAN)
    rp_prune["kernels"] = "k_tb_light + k_tb_heavy (four tiers), run concurrently"
    rp_prune["entries_examined"] = prune_stats["wedges"]
    rp_prune["entries_examined_per_s"] = round(prune_stats["wedges"] / (prune_ms * 1e-3), 1)
    res = {
        "gteps": mcc / (ms_step * 1e-3) / 1e9,
        "ms_per_step": ms_step,
        "solve_only_gteps": mcc / (solve_ms * 1e-3) / 1e9,
        "prune_ms": prune_ms, "solve_ms": solve_ms,
        "trials": {"n": len(pr), "prune_main_ms_mean": prune_ms,
                   "prune_main_ms_median": float(np.median(pr)),
                   "solve_kernel_ms_mean": solve_ms, "solve_kernel_ms_median": float(np.median(so)),
                   "step_ms_mean": float(np.mean(whole)), "step_ms_median": float(np.median(whole)),
                   "mall_flushed": True},
        "n": g.n, "m": g.m, "m_kept": kept_m, "m_cc": mcc, "reached": reached, "source": s,
        "stats": st,
        "roofline_solve": roofline("k_solve", b_solve, solve_ms, workload="rmat20"),
        "roofline_prune": rp_prune,
        "prune_stats": {"edges_pruned": prune_stats["edges_pruned"],
                        "hub_pass_deleted": prune_stats["hub_pruned"],
                        "entries_examined": prune_stats["wedges"]},
        "autotune": autotune_res,
    }
    if cpu_leg:
        res["cpu_baseline"] = cpu_baseline_rmat20(g, s, mcc)
    return res


def cpu_baseline_rmat20(g, s, mcc):
    """The oracle as it stands on the host cores: mark-array Trishla (OpenMP,
    all threads) on the whole graph, then binary-heap Dijkstra (one thread)."""
    import oracle

    threads = oracle.max_threads()
    t0 = time.perf_counter()
    keep = oracle.trishla(g.row_ptr, g.col, g.w)
    t1 = time.perf_counter()
    src = g.src()[keep.astype(bool)]
    from paper_2103_12012_amd import gen

    gp = gen.from_arcs(g.n, src, g.col[keep.astype(bool)], g.w[keep.astype(bool)])
    t2 = time.perf_counter()
    oracle.sssp(gp.row_ptr, gp.col, gp.w, s)
    t3 = time.perf_counter()
    step = (t1 - t0) + (t3 - t2)
    return {"value": round(mcc / step / 1e9, 5), "unit": "GTEPS", "cores": threads,
            "kind": "oracle", "host": host_cpu(),
            "sample": f"one full step on the same R-MAT 20 graph: Trishla mark-array on "
                      f"{threads} threads {t1-t0:.2f}s + Dijkstra 1 thread {t3-t2:.2f}s"}


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0))}


# ------------------------------------------------------------------ extras
def b_solve(n, reached, m_r):
    """Algorithmic bytes of one solve: init 8 B and epilogue 16 B per vertex,
    row bounds + own label per reached vertex, col + cost + head label per
    arc out of a reached vertex."""
    return 24 * n + 16 * reached + 16 * m_r


def solve_bytes_from_dist(g, dist_u32_or_f32):
    reached_mask = (dist_u32_or_f32 != 0xFFFFFFFF) if dist_u32_or_f32.dtype == np.uint32 \
        else np.isfinite(dist_u32_or_f32)
    m_r = int(g.out_degree()[reached_mask].sum())
    return b_solve(g.n, int(reached_mask.sum()), m_r), int(reached_mask.sum()), m_r


def time_oracle_dijkstra(g, sources):
    """Single-thread oracle Dijkstra from each source; returns (seconds, dists)."""
    import oracle

    t0 = time.perf_counter()
    ds = [oracle.sssp(g.row_ptr, g.col, g.w, int(s)) for s in sources]
    return time.perf_counter() - t0, ds


def bench_grid(steps, cpu_leg=True):
    import torch

    from paper_2103_12012_amd import gen, sssp

    g = gen.grid(4096, 4096, seed=3)
    rp, c, w = sssp.to_device(g, "cuda")
    # the library defaults: the automatic options tried best in sweeps of
    # delta, P, lag, workgroup and grid size on this graph
    solver = sssp.Solver(rp, c, w, validate=False, stats=True, no_autotune=True)
    solver(0)
    torch.cuda.synchronize()
    ev = HipEvents()
    ts = []
    for _ in range(max(1, steps)):
        e = ev.pair()
        solver(0, events=e)
        ts.append(ev.ms(e))
    ms = float(np.mean(ts))
    st = solver.stats.read()
    dist = solver.dist.cpu().numpy().view(np.uint32)
    b, reached, m_r = solve_bytes_from_dist(g, dist)
    out = {"workload": "grid4096_corner", "n": g.n, "m": g.m, "solve_ms": ms,
           "solve_ms_median": float(np.median(ts)), "trials": len(ts),
           "gteps": g.m / (ms * 1e-3) / 1e9,
           "roofline": roofline("k_solve", b, ms, workload="grid4096"), "stats": st}
    if cpu_leg:
        import oracle

        secs, (d_ref,) = time_oracle_dijkstra(g, [0])
        out["matches_oracle"] = bool(np.array_equal(d_ref.astype(np.uint32), dist))
        out["cpu_baseline"] = {"value": round(g.m / secs / 1e9, 5), "unit": "GTEPS", "cores": 1,
                               "kind": "oracle", "host": host_cpu(),
                               "sample": f"the whole workload: binary-heap Dijkstra from the "
                                         f"corner, one thread, {secs:.2f}s"}
    return out


def bench_batch(steps, cpu_leg=True):
    import torch

    from paper_2103_12012_amd import gen, sssp

    rng = np.random.default_rng(4)
    scales = rng.integers(12, 19, size=64)
    graphs = [gen.rmat(int(sc), 4000 + i) for i, sc in enumerate(scales)]
    sg, ss = [], []
    for i, g in enumerate(graphs):
        for s in gen.random_sources(g, 4, 5000 + i):
            sg.append(i)
            ss.append(int(s))
    dg = [sssp.to_device(g, "cuda") for g in graphs]
    mcc = 0
    for gi, s in zip(sg, ss):
        mcc += m_reached(graphs[gi], s)[0]
    # the same 256 solves as single-source calls, each autotuned per scale
    tuned = {}
    for gi, s in zip(sg, ss):
        sc = int(scales[gi])
        if sc not in tuned:
            tuned[sc] = sssp.autotune(*dg[gi], s)
    solvers = {}
    for gi in set(sg):
        solvers[gi] = sssp.Solver(*dg[gi], validate=False)
    for gi, s in zip(sg, ss):
        solvers[gi](s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for gi, s in zip(sg, ss):
            solvers[gi](s)
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t0) / steps * 1e3
    # the batched launch, tuned as a whole (sssp_autotune_batch), replayed
    # from a captured HIP graph
    b = sssp.BatchSolver(dg, sg, ss)
    tuned_batch = b.autotune()
    b()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            b()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) / steps * 1e3
    # algorithmic bytes of the 256 solves, from the batched output
    dists = [d.cpu().numpy().view(np.uint32) for d in b.split(b.dist)]
    b_total = 0
    for gi, d in zip(sg, dists):
        b_total += solve_bytes_from_dist(graphs[gi], d)[0]
    # k_solve of the batched launch alone (HIP events around it), eager; the
    # last two k_solve dispatches of this leg (the counter profile reads them)
    ev = HipEvents()
    kms = []
    for _ in range(2):
        e = ev.pair()
        b(events=e)
        kms.append(ev.ms(e))
    kernel_ms = float(np.mean(kms))
    out = {"workload": "batched_64rmat_12to18_x4", "solves": len(sg), "m_cc_total": mcc,
           "tuned_batch": tuned_batch,
           "tuned_single": {str(k): v for k, v in sorted(tuned.items())},
           "batch_ms": batch_ms, "batch_gteps": mcc / (batch_ms * 1e-3) / 1e9,
           "batch_k_solve_ms": kernel_ms,
           "single_calls_ms": single_ms, "single_gteps": mcc / (single_ms * 1e-3) / 1e9,
           "roofline_batched": roofline("k_solve", b_total, kernel_ms, workload="batch"),
           "roofline_single_calls": roofline("256 sssp_solve calls", b_total, single_ms)}
    out["roofline_single_calls"]["note"] = ("whole-call time of the 256 calls (launch gaps "
                                            "included), same algorithmic bytes")
    if cpu_leg:
        # bounded sample: the first source of each of the 64 graphs
        pick = [k for k in range(len(sg)) if k % 4 == 0]
        secs = 0.0
        m_sample = 0
        ok = True
        for k in pick:
            g = graphs[sg[k]]
            t, (d_ref,) = time_oracle_dijkstra(g, [ss[k]])
            secs += t
            m_sample += m_reached(g, ss[k])[0]
            ok = ok and np.array_equal(np.where(d_ref == np.iinfo(np.uint64).max, 0xFFFFFFFF,
                                                d_ref).astype(np.uint32), dists[k])
        out["sample_matches_oracle"] = bool(ok)
        out["cpu_baseline"] = {"value": round(m_sample / secs / 1e9, 5), "unit": "GTEPS",
                               "cores": 1, "kind": "oracle", "host": host_cpu(),
                               "sample": f"64 of the 256 solves (the first source of every "
                                         f"graph), binary-heap Dijkstra one thread, "
                                         f"{secs:.2f}s"}
    return out


def b_bwd(n, m, reached):
    """Algorithmic bytes of the backward: clear grad_w (4 B per arc), read
    dist, pred_edge and the upstream gradient and keep a subtree total per
    vertex (20 B), scatter one gradient per reached vertex (4 B)."""
    return 4 * m + 20 * n + 4 * reached


def bench_diff(steps, cpu_leg=True):
    import torch

    from paper_2103_12012_amd import gen, sssp

    g = gen.rmat(22, 22, weight="f32", wlo=0.5, whi=1.5)
    s = int(gen.random_sources(g, 1, 22)[0])
    t = gen.random_targets(g, s, 1024, 23)
    mcc, ncc = m_reached(g, s)
    rp, c, w = sssp.to_device(g, "cuda")
    gd = torch.zeros(g.n, dtype=torch.float32, device="cuda")
    gd[torch.from_numpy(t).long().cuda()] = 1.0
    solver = sssp.Solver(rp, c, w, validate=False, want_pred=False)
    solver(s)
    ev = HipEvents()
    L = sssp.lib()
    gcsr = sssp._csr(rp, c, w)
    o = sssp.make_opts(validate=False)
    nb = ctypes.c_size_t(0)
    assert L.sssp_backward(ctypes.byref(gcsr), s, None, None, None, None, ctypes.byref(o),
                           None, None, ctypes.byref(nb), None) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    grad_w = torch.empty(g.m, dtype=torch.float32, device="cuda")
    bst = sssp.StatsBuffer.new("cuda")
    fwd, bwd = [], []
    for _ in range(max(1, steps)):
        e1 = ev.pair()
        solver(s, events=e1)
        e2 = ev.pair()
        o2 = sssp.Opts.from_buffer_copy(o)
        o2.event_start, o2.event_stop = e2
        n2 = ctypes.c_size_t(ws.numel())
        rc = L.sssp_backward(ctypes.byref(gcsr), s, sssp._ptr(solver.dist),
                             sssp._ptr(solver.pred_edge), sssp._ptr(gd), sssp._ptr(grad_w),
                             ctypes.byref(o2), sssp._ptr(bst.t), sssp._ptr(ws), ctypes.byref(n2),
                             sssp._stream())
        assert rc == 0
        fwd.append(ev.ms(e1))
        bwd.append(ev.ms(e2))
    torch.cuda.synchronize()
    status = bst.read()["status"]
    fwd_ms, bwd_ms = float(np.mean(fwd)), float(np.mean(bwd))
    dist = solver.dist.cpu().numpy()
    gw = grad_w.cpu().numpy()
    bf, reached, m_r = solve_bytes_from_dist(g, dist)
    out = {"workload": "rmat22_f32_1024_targets", "n": g.n, "m": g.m, "m_cc": mcc,
           "forward_ms": fwd_ms, "backward_ms": bwd_ms, "backward_status": status,
           "forward_gteps": mcc / (fwd_ms * 1e-3) / 1e9,
           "roofline_forward": roofline("k_solve", bf, fwd_ms, workload="rmat22f32"),
           "roofline_backward": roofline("k_bwd", b_bwd(g.n, g.m, reached), bwd_ms,
                                         workload="rmat22f32"),
           "trials": len(fwd)}
    out["roofline_backward"]["kernels"] = "every kernel of sssp_backward (HIP events around them)"
    # the plain single-source kernel on the same topology with uint32 costs
    gu = gen.rmat(22, 22)
    assert np.array_equal(gu.col, g.col)
    rpu, cu, wu = sssp.to_device(gu, "cuda")
    su = sssp.Solver(rpu, cu, wu, validate=False, want_pred=False)
    su(s)
    us = []
    for _ in range(max(1, steps)):
        e = ev.pair()
        su(s, events=e)
        us.append(ev.ms(e))
    # same topology, so the same arcs are reached (m_cc)
    out["u32_same_graph"] = {"weights": "uint32 U{1..255}", "solve_ms": float(np.mean(us)),
                             "gteps": mcc / (float(np.mean(us)) * 1e-3) / 1e9}
    del gu, rpu, cu, wu, su
    if cpu_leg:
        import oracle

        t0 = time.perf_counter()
        d_ref = oracle.sssp(g.row_ptr, g.col, g.w, s)
        t1 = time.perf_counter()
        pe_ref, _ = oracle.pred(g.row_ptr, g.col, g.w, s, d_ref)
        gv = np.zeros(g.n, np.float32)
        gv[t] = 1.0
        t2 = time.perf_counter()
        g_ref = oracle.grad(g.row_ptr, s, pe_ref, gv)
        t3 = time.perf_counter()
        nz = g_ref != 0
        rel = np.abs(gw[nz] - g_ref[nz]) / np.abs(g_ref[nz])
        out["check"] = {
            "dist_bitwise_mismatches": int((dist.view(np.uint32) != d_ref.view(np.uint32)).sum()),
            "grad_max_rel_err": float(rel.max()) if rel.size else 0.0,
            "grad_max_abs_err_where_ref_zero": float(np.abs(gw[~nz]).max()) if (~nz).any() else 0.0,
            "grad_nonzero_arcs": int(nz.sum()), "tolerance_rel": 1e-4}
        out["cpu_baseline"] = {"value": round(mcc / (t1 - t0) / 1e9, 5), "unit": "GTEPS",
                               "cores": 1, "kind": "oracle", "host": host_cpu(),
                               "backward_ms": round((t3 - t2) * 1e3 + (t2 - t1) * 1e3, 2),
                               "sample": f"the whole workload: fp32 binary-heap Dijkstra "
                                         f"{t1-t0:.2f}s, then predecessor pass {t2-t1:.2f}s and "
                                         f"tree-path gradient {t3-t2:.3f}s, one thread"}
    return out


def bench_ablation(steps):
    """Local rule ablation on the pruned R-MAT 20 graph (256 partitions): the
    bucket width decides how literally each partition follows Alg. 3.
    delta = 1 on integer costs settles every partition in exact distance
    order (a bucket queue: the local Dijkstra order), delta = -1 is one
    unbounded bucket (fully asynchronous Bellman-Ford), 0 is the automatic
    width.  Same graph, source and partitions as the headline step."""
    import torch

    from paper_2103_12012_amd import gen, sssp

    g = gen.rmat(20, 20)
    s = int(gen.random_sources(g, 1, 20)[0])
    rp, c, w = sssp.to_device(g, "cuda")
    keep, (prp, pc, pw, emap) = sssp.prune(rp, c, w, num_partitions=256, validate=False)
    torch.cuda.synchronize()
    kept = int(prp[-1].item())
    ev = HipEvents()
    out = {"workload": "rmat20_pruned_local_rule", "partitions": 256}
    rows = (("dijkstra_order_delta1", dict(delta=1.0, lag=-1)),
            ("dijkstra_order_delta1_lag1", dict(delta=1.0, lag=1)),
            ("async_bellman_ford", dict(delta=-1.0)),
            ("auto", {}),
            # Alg. 3 literally: one vertex at a time from an LDS binary heap
            ("dijkstra_heap", dict(local_heap=True)),
            ("dijkstra_heap_unbounded_lag", dict(local_heap=True, lag=-1)),
            # cross-partition updates buffered per head in LDS (future-work buffering)
            ("buffered_cross_updates", dict(buffer_cross=True)))
    for name, kw in rows:
        solver = sssp.Solver(prp, pc[:kept], pw[:kept], num_partitions=256, validate=False,
                             stats=True, no_autotune=True, **kw)
        ts = []
        for _ in range(max(2, steps)):
            e = ev.pair()
            solver(s, events=e)
            ts.append(ev.ms(e))
        st = solver.stats.read()
        out[name] = {"solve_ms": float(np.median(ts)), "edges_relaxed": st["edges_relaxed"],
                     "label_updates": st["label_updates"],
                     "vertices_expanded": st["vertices_expanded"], "batches": st["batches"]}
    # Trishla with and without its hub pass (the same deletion set): the scan
    # phase (library events) and the whole prune call (stream events)
    for name, hubs in (("prune_with_hub_pass", True), ("prune_without_hub_pass", False)):
        scan, whole = [], []
        for _ in range(max(3, steps)):
            st_buf = sssp.StatsBuffer.new("cuda")
            e = ev.pair()
            t0e = torch.cuda.Event(enable_timing=True)
            t1e = torch.cuda.Event(enable_timing=True)
            t0e.record()
            sssp.prune(rp, c, w, compact=False, num_partitions=256, validate=False, sync=False,
                       stats=st_buf, events=e, hubs=hubs)
            t1e.record()
            torch.cuda.synchronize()
            scan.append(ev.ms(e))
            whole.append(t0e.elapsed_time(t1e))
        pst = st_buf.read()
        out[name] = {"scan_ms": float(np.median(scan)), "prune_call_ms": float(np.median(whole)),
                     "entries_examined": pst["wedges"], "hub_pass_deleted": pst["hub_pruned"],
                     "edges_pruned": pst["edges_pruned"]}
    # idle-time LOCAL pruning inside the solve, on the unpruned graph (no
    # separate Trishla phase), against the plain solve of the unpruned graph
    for name, kw in (("unpruned_plain", {}), ("unpruned_idle_prune", dict(idle_prune=True))):
        solver = sssp.Solver(rp, c, w, num_partitions=256, validate=False, stats=True,
                             no_autotune=True, **kw)
        ts = []
        for _ in range(max(2, steps)):
            e = ev.pair()
            solver(s, events=e)
            ts.append(ev.ms(e))
        st = solver.stats.read()
        out[name] = {"solve_ms": float(np.median(ts)), "edges_relaxed": st["edges_relaxed"],
                     "edges_pruned_during_solve": st["edges_pruned"],
                     "two_arc_paths_examined": st["wedges"]}
    return out


def bench_copy(steps):
    """A plain device copy of 1 GiB: the calibration that scales the
    FETCH_SIZE / WRITE_SIZE counters to bytes (each reads 1 GiB ideally)."""
    import torch

    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.copy_(a)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    return {"workload": "device_copy_1GiB", "bytes_read": n, "bytes_written": n,
            "ms": ms, "gbs": 2 * n / (ms * 1e-3) / 1e9}


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only", nargs="*", default=None,
                    help="subset of: rmat20 grid batch diff ablation copy (copy: counter "
                         "calibration, not part of the default run)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--skip-autotune", action="store_true",
                    help="headline: skip the autotune comparison (counter runs: every solve "
                         "of the leg then uses the default options)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus 1): the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    only = set(args.only) if args.only else {"rmat20", "grid", "batch", "diff", "ablation"}
    extra = {}
    head = None
    if "rmat20" in only:
        head = bench_rmat20(args.steps, args.warmup, cpu_leg=not args.no_cpu,
                            tune=not args.skip_autotune)
        print(f"[bench] rmat20 done: {head['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)
    for name, fn in (("grid", bench_grid), ("batch", bench_batch), ("diff", bench_diff),
                     ("ablation", bench_ablation), ("copy", bench_copy)):
        if name in only:
            k = max(1, min(args.steps, 5))
            extra[name] = fn(k, cpu_leg=not args.no_cpu) if name in ("grid", "batch", "diff") \
                else fn(k)
            print(f"[bench] {name} done", file=sys.stderr, flush=True)
    line = {"metric": METRIC, "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic"}
    if head is not None:
        # the roofline names the dominant part of the step: the Trishla scan
        # phase (five kernels run concurrently; the big tier's kernel spans the
        # phase, see profiles/k_solve_trishla_rmat20_step.txt); the solve's
        # own kernel is reported beside it as roofline_solve
        dom = head["roofline_prune"]
        line.update({
            "value": round(head["gteps"], 4), "ms_per_step": round(head["ms_per_step"], 4),
            "config": {"workload": "rmat20_trishla_then_sssp", "scale": 20, "edge_factor": 16,
                       "abcd": [0.57, 0.19, 0.19, 0.05], "weights": "uint32 U{1..255}",
                       "n": head["n"], "m": head["m"], "m_kept": head["m_kept"],
                       "partitions": 256, "source": head["source"], "m_cc": head["m_cc"]},
            "roofline": dom,
            "solve_only_gteps": round(head["solve_only_gteps"], 4),
            "prune_ms": round(head["prune_ms"], 4), "solve_ms": round(head["solve_ms"], 4),
            "trials": head["trials"],
            "roofline_solve": head["roofline_solve"], "roofline_prune": head["roofline_prune"],
            "solve_stats": head["stats"], "prune_stats": head["prune_stats"],
            "autotune": head["autotune"],
        })
        if "cpu_baseline" in head:
            line["cpu_baseline"] = head["cpu_baseline"]
    else:
        line.update({"value": None, "ms_per_step": None, "config": {"workload": "extras"}})
    line["extra"] = extra
    print(json.dumps(line))


if __name__ == "__main__":
    main()
