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
def bench_rmat20(steps, warmup, cpu_leg=True):
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
    solver = sssp.Solver(out_rp, out_c[:kept_m], out_w[:kept_m], num_partitions=P,
                         validate=False, stats=True)
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
        "roofline_prune": roofline("k_tb_light+k_tb_heavy", b_prune, prune_ms, workload="rmat20",
                                   parts=TRISHLA_SCAN),
        "wedges": st.get("wedges"),
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
def bench_grid(steps):
    import torch

    from paper_2103_12012_amd import gen, sssp

    g = gen.grid(4096, 4096, seed=3)
    rp, c, w = sssp.to_device(g, "cuda")
    solver = sssp.Solver(rp, c, w, validate=False, stats=True)
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
    b = 24 * g.n + 16 * g.n + 16 * g.m
    return {"workload": "grid4096_corner", "n": g.n, "m": g.m, "solve_ms": ms,
            "gteps": g.m / (ms * 1e-3) / 1e9, "roofline": roofline("k_solve", b, ms),
            "stats": st}


def bench_batch(steps):
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
    # the batched launch is tuned as a whole (sssp_autotune_batch); the single
    # calls below use per-scale single-solve tuning (sssp_autotune)
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
    return {"workload": "batched_64rmat_12to18_x4", "solves": len(sg), "m_cc_total": mcc,
            "tuned_batch": tuned_batch,
            "tuned_single": {str(k): v for k, v in sorted(tuned.items())},
            "batch_ms": batch_ms, "batch_gteps": mcc / (batch_ms * 1e-3) / 1e9,
            "single_calls_ms": single_ms, "single_gteps": mcc / (single_ms * 1e-3) / 1e9}


def bench_diff(steps):
    import torch

    from paper_2103_12012_amd import gen, sssp

    g = gen.rmat(22, 22, weight="f32", wlo=0.5, whi=1.5)
    s = int(gen.random_sources(g, 1, 22)[0])
    t = gen.random_targets(g, s, 1024, 23)
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
                             ctypes.byref(o2), None, sssp._ptr(ws), ctypes.byref(n2),
                             sssp._stream())
        assert rc == 0
        fwd.append(ev.ms(e1))
        bwd.append(ev.ms(e2))
    return {"workload": "rmat22_f32_1024_targets", "n": g.n, "m": g.m,
            "forward_ms": float(np.mean(fwd)), "backward_ms": float(np.mean(bwd)),
            "tolerance": "1e-5 rel dist (bit-exact expected), 1e-4 grad"}


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
    for name, delta, lag in (("dijkstra_order_delta1", 1.0, -1), ("dijkstra_order_delta1_lag1", 1.0, 1),
                             ("async_bellman_ford", -1.0, 0), ("auto", 0.0, 0)):
        solver = sssp.Solver(prp, pc[:kept], pw[:kept], num_partitions=256, delta=delta,
                             lag=lag, validate=False, stats=True, no_autotune=True)
        ts = []
        for _ in range(max(2, steps)):
            e = ev.pair()
            solver(s, events=e)
            ts.append(ev.ms(e))
        st = solver.stats.read()
        out[name] = {"solve_ms": float(np.median(ts)), "edges_relaxed": st["edges_relaxed"],
                     "label_updates": st["label_updates"],
                     "vertices_expanded": st["vertices_expanded"], "batches": st["batches"]}
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
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
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
        head = bench_rmat20(args.steps, args.warmup, cpu_leg=not args.no_cpu)
        print(f"[bench] rmat20 done: {head['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)
    for name, fn in (("grid", bench_grid), ("batch", bench_batch), ("diff", bench_diff),
                     ("ablation", bench_ablation), ("copy", bench_copy)):
        if name in only:
            extra[name] = fn(max(1, min(args.steps, 5)))
            print(f"[bench] {name} done", file=sys.stderr, flush=True)
    line = {"metric": METRIC, "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic"}
    if head is not None:
        # the roofline names k_solve, the longest kernel that has the GPU to
        # itself; the Trishla scan phase (reported as roofline_prune) is five
        # kernels run concurrently on four streams, so no single one of them
        # owns its launch time (see profiles/k_solve_trishla_rmat20_step.txt)
        dom = head["roofline_solve"]
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
            "solve_stats": head["stats"],
        })
        if "cpu_baseline" in head:
            line["cpu_baseline"] = head["cpu_baseline"]
    else:
        line.update({"value": None, "ms_per_step": None, "config": {"workload": "extras"}})
    line["extra"] = extra
    print(json.dumps(line))


if __name__ == "__main__":
    main()
