"""CPU oracle for single-source shortest paths with Trishla pruning.

TEST INFRASTRUCTURE ONLY: the checker the HIP library is compared against.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It imports nothing from the GPU library, and the GPU
library never imports it.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc); this module
only marshals numpy arrays.  Each function cites the passage of the paper it
follows:

* ``sssp``            Sec. I problem statement; Sec. III-C, Alg. 3 (Dijkstra)
* ``bellman_ford``    Sec. II / III-C (Bellman-Ford), brute force, tiny graphs
* ``pred``            tie rule for the shortest-path tree (paper silent)
* ``trishla``         Sec. III-B, Alg. 1 (brute force and mark-array forms)
* ``certify``         dual of the Sec. I path LP (feasible + tight tree)
* ``grad``            gradient of sum g[v] d(v) along the tree (not in paper)
* ``finite_diff``     float64 central differences of the same loss
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

U32_INF = 0xFFFFFFFF

CERT_CODES = {
    0: "ok", 1: "source", 2: "infeasible arc", 3: "unreached with pred",
    4: "pred not an arc into v", 5: "pred arc not tight",
    6: "smaller tight arc exists", 7: "pred chain does not reach source",
    8: "out of memory",
}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.oracle_certify_u32.restype = ctypes.c_int
        _lib.oracle_certify_f32.restype = ctypes.c_int
    return _lib


def max_threads() -> int:
    """Threads the OpenMP routines (Trishla) run on."""
    return int(_load().oracle_max_threads())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _graph(row_ptr, col, w):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w)
    n = rp.shape[0] - 1
    assert rp[0] == 0 and rp[-1] == c.shape[0] == w.shape[0]
    return n, rp, c, w


def _kind(w: np.ndarray) -> str:
    if w.dtype == np.uint32:
        return "u32"
    if w.dtype == np.float32:
        return "f32"
    if w.dtype == np.float64:
        return "f64"
    raise TypeError(f"weights must be uint32, float32 or float64, got {w.dtype}")


def sssp(row_ptr, col, w, source: int):
    """Binary-heap Dijkstra.  Returns dist: uint64 (UINT64_MAX = unreached) for
    uint32 weights, float32 / float64 (+inf = unreached) otherwise."""
    lib = _load()
    n, rp, c, w = _graph(row_ptr, col, w)
    k = _kind(w)
    if k == "u32":
        d = np.empty(n, dtype=np.uint64)
        rc = lib.oracle_sssp_u32(n, _p(rp), _p(c), _p(w), int(source), _p(d))
    elif k == "f32":
        d = np.empty(n, dtype=np.float32)
        rc = lib.oracle_sssp_f32(n, _p(rp), _p(c), _p(w), int(source), _p(d))
    else:
        d = np.empty(n, dtype=np.float64)
        rc = lib.oracle_sssp_f64(n, _p(rp), _p(c), _p(w), int(source), _p(d))
    if rc != 0:
        raise MemoryError("oracle_sssp")
    return d


def bellman_ford(row_ptr, col, w, source: int):
    """Brute-force Bellman-Ford (sweeps until nothing changes)."""
    lib = _load()
    n, rp, c, w = _graph(row_ptr, col, w)
    k = _kind(w)
    if k == "u32":
        d = np.empty(n, dtype=np.uint64)
        rc = lib.oracle_bellman_ford_u32(n, _p(rp), _p(c), _p(w), int(source), _p(d))
    elif k == "f32":
        d = np.empty(n, dtype=np.float32)
        rc = lib.oracle_bellman_ford_f32(n, _p(rp), _p(c), _p(w), int(source), _p(d))
    else:
        raise TypeError("bellman_ford supports uint32 and float32 weights")
    assert rc == 0
    return d


def pred(row_ptr, col, w, source: int, dist):
    """(pred_edge, pred): smallest tight edge id into every reached v != source."""
    lib = _load()
    n, rp, c, w = _graph(row_ptr, col, w)
    pe = np.empty(n, dtype=np.int32)
    pv = np.empty(n, dtype=np.int32)
    k = _kind(w)
    fn = {"u32": lib.oracle_pred_u32, "f32": lib.oracle_pred_f32,
          "f64": lib.oracle_pred_f64}[k]
    want = {"u32": np.uint64, "f32": np.float32, "f64": np.float64}[k]
    d = np.ascontiguousarray(dist, dtype=want)
    fn(n, _p(rp), _p(c), _p(w), int(source), _p(d), _p(pe), _p(pv))
    return pe, pv


def solve(row_ptr, col, w, source: int):
    """Oracle result in the library's output convention.

    Returns (dist, pred, pred_edge) with dist uint32 (0xFFFFFFFF unreached) for
    integer weights -- raising OverflowError if a distance reaches 2**32-1 --
    or float32 (+inf unreached) for fp32 weights -- raising OverflowError if a
    vertex reachable from the source has the float32 distance +inf (its path
    sum overflowed).  Only final distances decide: a path that overflows
    while a shorter one exists is no error.
    """
    d = sssp(row_ptr, col, w, source)
    pe, pv = pred(row_ptr, col, w, source, d)
    if d.dtype == np.uint64:
        reached = d != np.iinfo(np.uint64).max
        if reached.any() and d[reached].max() >= U32_INF:
            raise OverflowError("distance does not fit uint32")
        out = np.full(d.shape, U32_INF, dtype=np.uint32)
        out[reached] = d[reached].astype(np.uint32)
        d = out
    elif d.dtype == np.float32 and not np.isfinite(d).all():
        if reachable(row_ptr, col, source)[~np.isfinite(d)].any():
            raise OverflowError("a reachable vertex has distance +inf in float32")
    return d, pv, pe


def reachable(row_ptr, col, source: int):
    """Vertices reachable from ``source`` (breadth-first search by scipy)."""
    import scipy.sparse as sps
    from scipy.sparse.csgraph import breadth_first_order

    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    n = rp.shape[0] - 1
    a = sps.csr_matrix((np.ones(c.shape[0], dtype=np.int8), c, rp), shape=(n, n))
    order = breadth_first_order(a, int(source), directed=True, return_predecessors=False)
    mask = np.zeros(n, dtype=bool)
    mask[order] = True
    return mask


def trishla(row_ptr, col, w, local_scope: bool = False, nparts: int = 1,
            method: str = "mark"):
    """keep mask (uint8[m]) of Trishla pruning; method 'brute' or 'mark'."""
    lib = _load()
    n, rp, c, w = _graph(row_ptr, col, w)
    keep = np.empty(c.shape[0], dtype=np.uint8)
    k = _kind(w)
    if k not in ("u32", "f32"):
        raise TypeError("trishla supports uint32 and float32 weights")
    fn = getattr(lib, f"oracle_trishla_{method}_{k}")
    fn(n, _p(rp), _p(c), _p(w), int(bool(local_scope)), int(nparts), _p(keep))
    return keep


def certify(row_ptr, col, w, source: int, dist, pred_edge):
    """Check (dist, pred_edge) against the LP dual; returns (code, where)."""
    lib = _load()
    n, rp, c, w = _graph(row_ptr, col, w)
    pe = np.ascontiguousarray(pred_edge, dtype=np.int32)
    where = ctypes.c_int64(-1)
    if _kind(w) == "u32":
        d = np.ascontiguousarray(dist, dtype=np.uint32)
        rc = lib.oracle_certify_u32(n, _p(rp), _p(c), _p(w), int(source), _p(d),
                                    _p(pe), ctypes.byref(where))
    else:
        d = np.ascontiguousarray(dist, dtype=np.float32)
        rc = lib.oracle_certify_f32(n, _p(rp), _p(c), _p(w), int(source), _p(d),
                                    _p(pe), ctypes.byref(where))
    return int(rc), int(where.value)


def grad(row_ptr, source: int, pred_edge, g):
    """d(sum_v g[v] d(v)) / d w along the tree pred_edge (float32[m])."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    n = rp.shape[0] - 1
    pe = np.ascontiguousarray(pred_edge, dtype=np.int32)
    gg = np.ascontiguousarray(g, dtype=np.float32)
    out = np.empty(int(rp[-1]), dtype=np.float32)
    rc = lib.oracle_grad_f32(n, _p(rp), int(source), _p(pe), _p(gg), _p(out))
    if rc != 0:
        raise RuntimeError(f"oracle_grad_f32: {CERT_CODES.get(rc, rc)}")
    return out


def finite_diff(row_ptr, col, w, source: int, g, eps: float = 1e-3, edges=None):
    """Central differences of L(w) = sum g[v] d_w(v) in float64.

    Returns (fd, valid): fd[e] for the requested edges; valid[e] is False when
    the float64 shortest-path tree changes at w +- eps (the loss is not
    differentiable there), in which case fd[e] is not meaningful.
    """
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    w64 = np.ascontiguousarray(w, dtype=np.float64)
    g64 = np.asarray(g, dtype=np.float64)
    d0 = sssp(rp, c, w64, source)
    pe0, _ = pred(rp, c, w64, source, d0)
    m = c.shape[0]
    edges = np.arange(m) if edges is None else np.asarray(edges)
    fd = np.zeros(edges.shape[0], dtype=np.float64)
    valid = np.ones(edges.shape[0], dtype=bool)
    reach = np.isfinite(d0)
    for i, e in enumerate(edges):
        vals = []
        for s in (+1.0, -1.0):
            wp = w64.copy()
            wp[e] += s * eps
            d = sssp(rp, c, wp, source)
            pe, _ = pred(rp, c, wp, source, d)
            if not np.array_equal(pe, pe0):
                valid[i] = False
            vals.append(float(np.dot(g64[reach], d[reach])))
        fd[i] = (vals[0] - vals[1]) / (2 * eps)
    return fd, valid
