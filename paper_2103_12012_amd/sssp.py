"""Python binding of libsssp.so (the gfx950 HIP library), same names as the
C ABI in include/sssp.h: ``prune``, ``solve``, ``solve_batch``, ``backward``,
``autotune``, plus :class:`SSSPDist`, a ``torch.autograd.Function`` whose
backward calls ``sssp_backward``.

This module only marshals arguments: torch tensors supply device memory and
the current HIP stream; every step of the computation runs in the library's
kernels.  There is no CPU fallback: if the library is missing, ``lib()``
raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SSSP_LIB", os.path.join(_HERE, "libsssp.so"))
HEADER = os.path.join(_HERE, "..", "include", "sssp.h")

W_U32, W_F32 = 0, 1
F_VALIDATE, F_SYNC, F_PRUNE_LOCAL, F_NO_AUTOTUNE = 1, 2, 4, 8
F_BUFFER_CROSS, F_LOCAL_HEAP, F_IDLE_PRUNE, F_PRUNE_NO_HUBS = 16, 32, 64, 128

ERRORS = {
    0: "SSSP_OK", -1: "SSSP_ERR_ARG", -2: "SSSP_ERR_SOURCE", -3: "SSSP_ERR_CSR",
    -4: "SSSP_ERR_UNSORTED", -5: "SSSP_ERR_WEIGHT", -6: "SSSP_ERR_ZERO_WEIGHT",
    -7: "SSSP_ERR_OVERFLOW", -8: "SSSP_ERR_TIMEOUT", -9: "SSSP_ERR_WORKSPACE",
    -10: "SSSP_ERR_HIP", -11: "SSSP_ERR_CAPTURE", -12: "SSSP_ERR_CYCLE",
    -13: "SSSP_ERR_TOO_LARGE",
}
ERR_WORKSPACE = -9


class SSSPError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({strerror(code)})")


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("wtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("num_partitions", ctypes.c_int32),
                ("wg_size", ctypes.c_int32), ("num_workgroups", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("lag", ctypes.c_int32), ("event_start", ctypes.c_void_p),
                ("event_stop", ctypes.c_void_p), ("keep_out", ctypes.c_void_p)]


STATS_FIELDS = ["edges_relaxed", "label_updates", "cross_updates", "vertices_expanded",
                "batches", "edges_pruned", "wedges", "hub_pruned"]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("num_partitions", ctypes.c_int32),
                ("delta_bits", ctypes.c_uint64)] + \
               [(f, ctypes.c_uint64) for f in STATS_FIELDS] + \
               [("reserved", ctypes.c_uint64 * 5)]


_lib = None
_vp, _i32, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)


def lib() -> ctypes.CDLL:
    """Load libsssp.so (built by ``paper_2103_12012_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -m paper_2103_12012_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.sssp_strerror.restype = ctypes.c_char_p
        L.sssp_strerror.argtypes = [ctypes.c_int]
        L.sssp_version.restype = ctypes.c_char_p
        L.sssp_opts_init.argtypes = [P(Opts)]
        L.sssp_prune.argtypes = [P(CSR), P(Opts), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.sssp_solve.argtypes = [P(CSR), _i32, P(Opts), _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.sssp_solve_batch.argtypes = [_i32, P(CSR), _i32, P(_i32), P(_i32),
                                       P(ctypes.c_int64), P(Opts), _vp, _vp, _vp, _vp, _vp,
                                       _sz, _vp]
        L.sssp_backward.argtypes = [P(CSR), _i32, _vp, _vp, _vp, _vp, P(Opts), _vp, _vp, _sz,
                                    _vp]
        L.sssp_autotune.argtypes = [P(CSR), _i32, _vp, P(Opts), ctypes.c_char_p, _vp, _sz, _vp]
        L.sssp_autotune_batch.argtypes = [_i32, P(CSR), _i32, P(_i32), P(_i32),
                                          P(ctypes.c_int64), _vp, P(Opts), ctypes.c_char_p,
                                          _vp, _sz, _vp]
        L.sssp_solve_noalloc.argtypes = [P(CSR), _i32, P(Opts), _vp, _vp, _vp, _vp, _vp]
        for f in ("sssp_prune", "sssp_solve", "sssp_solve_batch", "sssp_backward",
                  "sssp_autotune", "sssp_autotune_batch", "sssp_solve_noalloc"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def declared_symbols() -> list[str]:
    """Function names declared in include/sssp.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(sssp_[a-z_]+)\s*\(", text)))


def strerror(code: int) -> str:
    return lib().sssp_strerror(int(code)).decode()


def version() -> str:
    return lib().sssp_version().decode()


def _check(rc: int, where: str):
    if rc != 0:
        raise SSSPError(rc, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _csr(row_ptr, col, w) -> CSR:
    for name, t in (("row_ptr", row_ptr), ("col", col)):
        if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous int32 device tensor")
    if w.dtype == torch.float32:
        wt = W_F32
    elif w.dtype in (torch.int32, torch.uint32):
        wt = W_U32
    else:
        raise TypeError("weights must be uint32 (or int32 bits) or float32")
    if not w.is_cuda or not w.is_contiguous():
        raise TypeError("w must be a contiguous device tensor")
    n = row_ptr.numel() - 1
    m = col.numel()
    if n < 1 or w.numel() != m:
        raise ValueError("row_ptr must have n+1 >= 2 entries and w as many as col")
    return CSR(n, m, row_ptr.data_ptr(), col.data_ptr() if m else None,
               w.data_ptr() if m else None, wt, 0)


def make_opts(delta=0.0, num_partitions=0, wg_size=0, num_workgroups=0, max_rounds=0,
              validate=True, sync=False, local=False, no_autotune=False, events=None,
              lag=0, buffer_cross=False, local_heap=False, idle_prune=False,
              hubs=True) -> Opts:
    flags = (F_VALIDATE if validate else 0) | (F_SYNC if sync else 0) | \
            (F_PRUNE_LOCAL if local else 0) | (F_NO_AUTOTUNE if no_autotune else 0) | \
            (F_BUFFER_CROSS if buffer_cross else 0) | (F_LOCAL_HEAP if local_heap else 0) | \
            (F_IDLE_PRUNE if idle_prune else 0) | (0 if hubs else F_PRUNE_NO_HUBS)
    o = Opts()
    o.delta = float(delta)
    o.num_partitions = int(num_partitions)
    o.wg_size = int(wg_size)
    o.num_workgroups = int(num_workgroups)
    o.max_rounds = int(max_rounds)
    o.flags = flags
    o.lag = int(lag)
    if events is not None:
        o.event_start, o.event_stop = events
    return o


def _workspace(query, device) -> torch.Tensor:
    nbytes = ctypes.c_size_t(0)
    _check(query(ctypes.byref(nbytes)), "workspace query")
    return torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=device)


@dataclass
class StatsBuffer:
    """Device-resident sssp_stats (read after the stream has finished)."""

    t: torch.Tensor

    @classmethod
    def new(cls, device):
        return cls(torch.zeros(ctypes.sizeof(Stats) // 8, dtype=torch.int64, device=device))

    def read(self) -> dict:
        raw = self.t.cpu().numpy().tobytes()
        s = Stats.from_buffer_copy(raw)
        out = {"status": s.status, "num_partitions": s.num_partitions,
               "delta_bits": int(s.delta_bits)}
        for f in STATS_FIELDS:
            out[f] = int(getattr(s, f))
        return out


# --------------------------------------------------------------------- prune
def prune(row_ptr, col, w, *, compact=True, local=False, num_partitions=0, validate=True,
          sync=True, stats=None, events=None, hubs=True):
    """Trishla pruning.  Returns keep (uint8[m]); with compact=True also
    (row_ptr', col', w', edge_map) of the kept arcs (trimmed, which reads the
    kept count back to the host).  hubs=False skips the hub pass (same
    result)."""
    g = _csr(row_ptr, col, w)
    o = make_opts(num_partitions=num_partitions, validate=validate, sync=sync, local=local,
                  events=events, hubs=hubs)
    dev = col.device
    L = lib()
    outs = (None,) * 4
    if compact:
        outs = (torch.empty(g.n + 1, dtype=torch.int32, device=dev),
                torch.empty(max(g.m, 1), dtype=torch.int32, device=dev),
                torch.empty(max(g.m, 1), dtype=w.dtype, device=dev),
                torch.empty(max(g.m, 1), dtype=torch.int32, device=dev))
    keep = torch.empty(max(g.m, 1), dtype=torch.uint8, device=dev)
    optr = [_ptr(t) for t in outs]
    ws = _workspace(lambda nb: L.sssp_prune(ctypes.byref(g), ctypes.byref(o), None, *optr,
                                            None, None, nb, None), dev)
    nb = ctypes.c_size_t(ws.numel())
    rc = L.sssp_prune(ctypes.byref(g), ctypes.byref(o), _ptr(keep), *optr,
                      _ptr(stats.t) if stats else None, _ptr(ws), ctypes.byref(nb), _stream())
    _check(rc, "sssp_prune")
    keep = keep[:g.m]
    if not compact:
        return keep
    rp, c2, w2, emap = outs
    mk = int(rp[-1].item())
    return keep, (rp, c2[:mk], w2[:mk], emap[:mk])


# --------------------------------------------------------------------- solve
class Solver:
    """A reusable single-source solve on one graph: the workspace and outputs
    are allocated once, so repeated calls (and HIP graph capture) allocate
    nothing."""

    def __init__(self, row_ptr, col, w, *, delta=0.0, num_partitions=0, wg_size=0,
                 num_workgroups=0, max_rounds=0, validate=True, want_pred=True,
                 stats=False, lag=0, no_autotune=False, buffer_cross=False,
                 local_heap=False, idle_prune=False, want_keep=False):
        self.g = _csr(row_ptr, col, w)
        self._keep = (row_ptr, col, w)
        self.opts = make_opts(delta, num_partitions, wg_size, num_workgroups, max_rounds,
                              validate=validate, lag=lag, no_autotune=no_autotune,
                              buffer_cross=buffer_cross, local_heap=local_heap,
                              idle_prune=idle_prune)
        # idle pruning: the keep flags of the arcs (1 kept, 0 deleted during the solve)
        self.keep = None
        if idle_prune and want_keep:
            self.keep = torch.empty(max(self.g.m, 1), dtype=torch.uint8, device=col.device)
            self.opts.keep_out = self.keep.data_ptr()
        dev = col.device
        self.col_device = dev
        n = self.g.n
        self.dist = torch.empty(n, dtype=w.dtype, device=dev)
        self.pred = torch.empty(n, dtype=torch.int32, device=dev) if want_pred else None
        self.pred_edge = torch.empty(n, dtype=torch.int32, device=dev)
        self.stats = StatsBuffer.new(dev) if stats else None
        L = lib()
        self.ws = _workspace(lambda nb: L.sssp_solve(ctypes.byref(self.g), 0,
                                                     ctypes.byref(self.opts), None, None,
                                                     None, None, None, nb, None), dev)

    def __call__(self, source: int, *, sync=False, events=None, validate=None):
        o = Opts.from_buffer_copy(self.opts)
        if sync:
            o.flags |= F_SYNC
        if validate is not None:
            o.flags = (o.flags | F_VALIDATE) if validate else (o.flags & ~F_VALIDATE)
        if events is not None:
            o.event_start, o.event_stop = events
        for attempt in range(2):
            nb = ctypes.c_size_t(self.ws.numel())
            rc = lib().sssp_solve(ctypes.byref(self.g), int(source), ctypes.byref(o),
                                  _ptr(self.dist), _ptr(self.pred), _ptr(self.pred_edge),
                                  _ptr(self.stats.t) if self.stats else None, _ptr(self.ws),
                                  ctypes.byref(nb), _stream())
            if rc != ERR_WORKSPACE or attempt:
                break
            # automatic options now resolve differently (the autotune cache
            # changed since construction): size the workspace again
            self.ws = _workspace(lambda q: lib().sssp_solve(
                ctypes.byref(self.g), 0, ctypes.byref(self.opts), None, None, None, None, None,
                q, None), self.col_device)
        _check(rc, "sssp_solve")
        return self.dist, self.pred, self.pred_edge


def solve(row_ptr, col, w, source: int, *, sync=True, **kw):
    """Single-source shortest paths.  Returns (dist, pred, pred_edge)."""
    s = Solver(row_ptr, col, w, **kw)
    return s(source, sync=sync)


# --------------------------------------------------------------- solve_batch
class BatchSolver:
    """Many (graph, source) solves in one persistent launch; the workspace and
    outputs are allocated once so the call can be captured and replayed."""

    def __init__(self, graphs, solve_graph, solve_source, *, delta=0.0, num_partitions=0,
                 wg_size=0, num_workgroups=0, validate=False, want_pred=True, stats=False,
                 buffer_cross=False, local_heap=False, idle_prune=False):
        self._keep = graphs
        self.gs = (CSR * len(graphs))(*[_csr(*g) for g in graphs])
        wdt = graphs[0][2].dtype
        dev = graphs[0][1].device
        self.solve_graph = (ctypes.c_int32 * len(solve_graph))(*[int(x) for x in solve_graph])
        self.solve_source = (ctypes.c_int32 * len(solve_source))(*[int(x) for x in solve_source])
        offs, tot = [], 0
        for gi in solve_graph:
            offs.append(tot)
            tot += self.gs[int(gi)].n
        self.offsets = offs
        self.out_offset = (ctypes.c_int64 * len(offs))(*offs)
        self.total = tot
        self.opts = make_opts(delta, num_partitions, wg_size, num_workgroups,
                              validate=validate, buffer_cross=buffer_cross,
                              local_heap=local_heap, idle_prune=idle_prune)
        self.dist = torch.empty(tot, dtype=wdt, device=dev)
        self.pred = torch.empty(tot, dtype=torch.int32, device=dev) if want_pred else None
        self.pred_edge = torch.empty(tot, dtype=torch.int32, device=dev)
        self.stats = StatsBuffer.new(dev) if stats else None
        L = lib()
        self.ws = _workspace(lambda nb: L.sssp_solve_batch(
            len(graphs), self.gs, len(solve_graph), self.solve_graph, self.solve_source,
            self.out_offset, ctypes.byref(self.opts), None, None, None, None, None, nb, None),
            dev)

    def __call__(self, *, sync=False, events=None):
        o = Opts.from_buffer_copy(self.opts)
        if sync:
            o.flags |= F_SYNC
        if events is not None:
            o.event_start, o.event_stop = events
        nb = ctypes.c_size_t(self.ws.numel())
        rc = lib().sssp_solve_batch(len(self._keep), self.gs, len(self.offsets),
                                    self.solve_graph, self.solve_source, self.out_offset,
                                    ctypes.byref(o), _ptr(self.dist), _ptr(self.pred),
                                    _ptr(self.pred_edge),
                                    _ptr(self.stats.t) if self.stats else None,
                                    _ptr(self.ws), ctypes.byref(nb), _stream())
        _check(rc, "sssp_solve_batch")
        return self.dist, self.pred, self.pred_edge

    def autotune(self, cache_path: str | None = None, **fixed) -> dict:
        """Tune this batched launch (sssp_autotune_batch); later automatic
        launches of batches with the same signature use the result.  The
        workspace is sized again for the tuned options."""
        L = lib()
        best = make_opts(validate=False, **fixed)
        args = (len(self._keep), self.gs, len(self.offsets), self.solve_graph, self.solve_source,
                self.out_offset)
        dev = self.dist.device
        ws = _workspace(lambda nb: L.sssp_autotune_batch(*args, None, ctypes.byref(best), None,
                                                         None, nb, None), dev)
        nb = ctypes.c_size_t(ws.numel())
        path = cache_path.encode() if cache_path else None
        rc = L.sssp_autotune_batch(*args, _ptr(self.dist), ctypes.byref(best), path, _ptr(ws),
                                   ctypes.byref(nb), _stream())
        _check(rc, "sssp_autotune_batch")
        del ws
        self.ws = _workspace(lambda q: L.sssp_solve_batch(
            *args, ctypes.byref(self.opts), None, None, None, None, None, q, None), dev)
        return {"delta": best.delta, "num_partitions": best.num_partitions,
                "wg_size": best.wg_size, "num_workgroups": best.num_workgroups}

    def split(self, t):
        """Per-solve views of a batched output tensor."""
        out = []
        for i, off in enumerate(self.offsets):
            n = self.gs[self.solve_graph[i]].n
            out.append(t[off:off + n])
        return out


def solve_batch(graphs, solve_graph, solve_source, *, sync=True, **kw):
    b = BatchSolver(graphs, solve_graph, solve_source, **kw)
    dist, pred, pe = b(sync=sync)
    return b.split(dist), (b.split(pred) if pred is not None else None), b.split(pe)


# ------------------------------------------------------------------ backward
def backward(row_ptr, col, w, source: int, dist, pred_edge, grad_dist, *, validate=True,
             sync=False, events=None, ws=None):
    """d(sum grad_dist * dist) / d w along the tree pred_edge (float32[m]).
    With sync=True a device-detected error raises SSSPError; the returned
    gradient is cleared to zero before any tree work, so after an error it
    holds zeros, never stale memory."""
    g = _csr(row_ptr, col, w)
    if g.wtype != W_F32:
        raise TypeError("backward needs float32 weights")
    o = make_opts(validate=validate, sync=sync, events=events)
    L = lib()
    dev = col.device
    if ws is None:
        ws = _workspace(lambda nb: L.sssp_backward(ctypes.byref(g), int(source), None, None,
                                                   None, None, ctypes.byref(o), None, None,
                                                   nb, None), dev)
    grad_w = torch.empty(max(g.m, 1), dtype=torch.float32, device=dev)
    nb = ctypes.c_size_t(ws.numel())
    gd = grad_dist.contiguous().to(torch.float32)
    rc = L.sssp_backward(ctypes.byref(g), int(source), _ptr(dist), _ptr(pred_edge), _ptr(gd),
                         _ptr(grad_w), ctypes.byref(o), None, _ptr(ws), ctypes.byref(nb),
                         _stream())
    _check(rc, "sssp_backward")
    return grad_w[:g.m]


class SSSPDist(torch.autograd.Function):
    """dist = SSSPDist.apply(w, row_ptr, col, source); gradients flow to w.

    Device-detected errors (an invalid or zero cost, an overflow, a time-out,
    a predecessor cycle) raise :class:`SSSPError` from forward and backward:
    both wait for their kernels and read the status word, except while the
    current stream is being captured into a graph (no synchronisation is
    allowed then; the caller checks the result)."""

    @staticmethod
    def forward(ctx, w, row_ptr, col, source):
        if w.dtype != torch.float32:
            raise TypeError("SSSPDist needs float32 weights")
        sync = not torch.cuda.is_current_stream_capturing()
        dist, _, pe = solve(row_ptr, col, w, int(source), sync=sync, want_pred=False)
        dist = dist.clone()
        pe = pe.clone()
        ctx.save_for_backward(w, row_ptr, col, dist, pe)
        ctx.source = int(source)
        return dist

    @staticmethod
    def backward(ctx, grad_dist):
        w, row_ptr, col, dist, pe = ctx.saved_tensors
        sync = not torch.cuda.is_current_stream_capturing()
        gw = backward(row_ptr, col, w, ctx.source, dist, pe, grad_dist, sync=sync)
        return gw, None, None, None


# ------------------------------------------------------------------ autotune
def autotune(row_ptr, col, w, source: int, cache_path: str | None = None, **fixed) -> dict:
    """Time candidate settings for this graph; the winner is cached in the
    library and returned as a dict of options.  Keyword arguments (delta,
    num_partitions, wg_size, num_workgroups, lag) fix those options."""
    g = _csr(row_ptr, col, w)
    L = lib()
    dev = col.device
    best = make_opts(validate=False, **fixed)
    ws = _workspace(lambda nb: L.sssp_autotune(ctypes.byref(g), int(source), None,
                                               ctypes.byref(best), None, None, nb, None), dev)
    scratch = torch.empty(g.n, dtype=torch.int32, device=dev)
    nb = ctypes.c_size_t(ws.numel())
    path = cache_path.encode() if cache_path else None
    rc = L.sssp_autotune(ctypes.byref(g), int(source), _ptr(scratch), ctypes.byref(best), path,
                         _ptr(ws), ctypes.byref(nb), _stream())
    _check(rc, "sssp_autotune")
    return {"delta": best.delta, "num_partitions": best.num_partitions,
            "wg_size": best.wg_size, "num_workgroups": best.num_workgroups, "lag": best.lag}


# ------------------------------------------------------------------ helpers
def to_device(g, device="cuda"):
    """Move a host CSR (paper_2103_12012_amd.gen.CSR) to device tensors."""
    import numpy as np

    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(device)
    c = torch.from_numpy(np.ascontiguousarray(g.col)).to(device)
    if g.w.dtype == np.uint32:
        w = torch.from_numpy(np.ascontiguousarray(g.w).view(np.int32)).to(device)
    else:
        w = torch.from_numpy(np.ascontiguousarray(g.w)).to(device)
    return rp, c, w
