"""Seeded synthetic graph inputs shared by the oracle tests and the GPU path.

This module only *draws inputs*: vertex pairs, weights, sources and targets,
laid out as CSR.  It performs none of the shortest-path or pruning arithmetic,
so both the CPU oracle and the HIP library can consume its output without
sharing any of the method's code.

The paper evaluates on synthetic graphs with uniformly drawn integer weights
(Sec. IV-A); the generators here stand in for those inputs:

* ``uniform``  -- directed uniform random arcs (no self-loops, duplicates kept);
* ``rmat``     -- recursive-matrix (R-MAT) power-law graphs, the published
                  quadrant-sampling method, deduplicated, self-loops removed;
* ``grid``     -- a 2D 4-neighbour grid, a road-like high-diameter graph.

Every graph is returned as a :class:`CSR` whose rows are sorted by column
(ties by weight, then by draw order), which is the layout the library expects.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

__all__ = [
    "CSR", "from_arcs", "uniform", "rmat", "grid", "random_sources",
    "reachable_mask", "random_targets", "weights_u32", "weights_f32",
]


@dataclasses.dataclass
class CSR:
    """A directed graph in compressed sparse row form (host numpy arrays).

    ``row_ptr`` is int32[n+1], ``col`` int32[m], ``w`` uint32[m] or float32[m].
    Edge id ``e`` is the position in ``col``; edges of row ``u`` are
    ``row_ptr[u] .. row_ptr[u+1]-1``.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def src(self) -> np.ndarray:
        """Tail vertex of every edge (int32[m])."""
        deg = np.diff(self.row_ptr.astype(np.int64))
        return np.repeat(np.arange(self.n, dtype=np.int32), deg)

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def with_weights(self, w: np.ndarray) -> "CSR":
        assert w.shape == self.col.shape
        return CSR(self.n, self.row_ptr, self.col, np.ascontiguousarray(w))

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        for a in (self.row_ptr, self.col, self.w):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def from_arcs(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray | None = None,
              dtype=np.uint32) -> CSR:
    """Build a CSR from arc arrays; rows sorted by (col, weight, draw order).

    When ``w`` is None the weights are left as zeros of ``dtype`` (callers draw
    them afterwards, in CSR order).
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if w is None:
        w = np.zeros(u.shape[0], dtype=dtype)
    w = np.asarray(w)
    if u.size:
        assert u.min() >= 0 and u.max() < n and v.min() >= 0 and v.max() < n
    order = np.lexsort((np.arange(u.shape[0]), w, v, u))
    u, v, w = u[order], v[order], w[order]
    counts = np.bincount(u, minlength=n) if u.size else np.zeros(n, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31 - 1
    return CSR(int(n), row_ptr.astype(np.int32), v.astype(np.int32),
               np.ascontiguousarray(w))


def weights_u32(rng: np.random.Generator, m: int, lo: int, hi: int) -> np.ndarray:
    """uint32 weights uniform on the integers {lo..hi}."""
    return rng.integers(lo, hi + 1, size=m, dtype=np.int64).astype(np.uint32)


def weights_f32(rng: np.random.Generator, m: int, lo: float, hi: float) -> np.ndarray:
    """float32 weights uniform on [lo, hi] (drawn in float64, rounded once)."""
    return rng.uniform(lo, hi, size=m).astype(np.float32)


def uniform(n: int, m: int, seed: int, wlo: int = 1, whi: int = 100) -> CSR:
    """Directed uniform random graph: m arcs, both endpoints uniform, u != v.

    The head is drawn from the n-1 vertices other than the tail.  Duplicate
    arcs are kept (each is its own edge instance).  Weights are uint32 uniform
    on {wlo..whi}, drawn together with the arcs.
    """
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n, size=m, dtype=np.int64)
    v = rng.integers(0, n - 1, size=m, dtype=np.int64)
    v = v + (v >= u)
    w = weights_u32(rng, m, wlo, whi)
    return from_arcs(n, u, v, w)


def _rmat_pairs(scale: int, m0: int, a: float, b: float, c: float,
                rng: np.random.Generator):
    """Draw m0 R-MAT (row, col) pairs by ``scale`` levels of quadrant choice.

    Quadrant a = (0,0), b = (0,1), c = (1,0), d = (1,1); the most significant
    bit is chosen first.  Thresholds are applied to 32-bit uniform integers.
    """
    ta = np.uint32(round(a * 2**32)) if a < 1 else np.uint32(2**32 - 1)
    tab = np.uint32(min(round((a + b) * 2**32), 2**32 - 1))
    tabc = np.uint32(min(round((a + b + c) * 2**32), 2**32 - 1))
    u = np.zeros(m0, dtype=np.uint32)
    v = np.zeros(m0, dtype=np.uint32)
    for _ in range(scale):
        r = rng.integers(0, 2**32, size=m0, dtype=np.uint32)
        row_bit = (r >= tab).astype(np.uint32)
        col_bit = (((r >= ta) & (r < tab)) | (r >= tabc)).astype(np.uint32)
        u <<= np.uint32(1)
        u |= row_bit
        v <<= np.uint32(1)
        v |= col_bit
        del r, row_bit, col_bit
    return u, v


def rmat(scale: int, seed: int, edge_factor: int = 16,
         abcd=(0.57, 0.19, 0.19, 0.05), weight="u32", wlo=1, whi=255) -> CSR:
    """R-MAT graph with 2**scale vertices and edge_factor * 2**scale drawn arcs.

    Self-loops and duplicate (u, v) pairs are removed before the weights are
    drawn; no vertex relabelling is applied, so hubs keep the lowest ids.
    ``weight`` is "u32" (uniform on {wlo..whi}) or "f32" (uniform on
    [wlo, whi]).
    """
    a, b, c, _d = abcd
    n = 1 << scale
    m0 = edge_factor * n
    rng = np.random.default_rng(seed)
    u, v = _rmat_pairs(scale, m0, a, b, c, rng)
    keep = u != v
    key = (u[keep].astype(np.uint64) << np.uint64(32)) | v[keep].astype(np.uint64)
    del u, v, keep
    key = np.unique(key)  # sorted by (u, v): already CSR order
    uu = (key >> np.uint64(32)).astype(np.int64)
    vv = (key & np.uint64(0xFFFFFFFF)).astype(np.int32)
    del key
    m = vv.shape[0]
    if weight == "u32":
        w = weights_u32(rng, m, int(wlo), int(whi))
    elif weight == "f32":
        w = weights_f32(rng, m, float(wlo), float(whi))
    else:
        raise ValueError(weight)
    counts = np.bincount(uu, minlength=n)
    del uu
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), vv, w)


def grid(rows: int, cols: int, seed: int, wlo: int = 1, whi: int = 1000,
         weight="u32") -> CSR:
    """rows x cols grid, id = r*cols + c, arcs to the 4 neighbours both ways.

    Every directed arc draws its own weight (so w(u->v) and w(v->u) differ in
    general).  Rows are in column order: up, left, right, down.
    """
    n = rows * cols
    deg = np.zeros(n, dtype=np.int64)
    idx = np.arange(n, dtype=np.int64)
    r, c = idx // cols, idx % cols
    has = [r > 0, c > 0, c < cols - 1, r < rows - 1]
    off = [-cols, -1, 1, cols]
    for h in has:
        deg += h
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    m = int(row_ptr[-1])
    col = np.empty(m, dtype=np.int32)
    pos = row_ptr[:-1].copy()
    for h, o in zip(has, off):
        sel = np.nonzero(h)[0]
        col[pos[sel]] = (sel + o).astype(np.int32)
        pos[sel] += 1
    del pos, r, c, idx
    rng = np.random.default_rng(seed)
    if weight == "u32":
        w = weights_u32(rng, m, wlo, whi)
    else:
        w = weights_f32(rng, m, float(wlo), float(whi))
    return CSR(n, row_ptr.astype(np.int32), col, w)


def random_sources(g: CSR, k: int, seed: int) -> np.ndarray:
    """k sources uniform over vertices with out-degree >= 1 (with replacement)."""
    rng = np.random.default_rng(seed)
    cand = np.nonzero(g.out_degree() > 0)[0]
    return rng.choice(cand, size=k, replace=True).astype(np.int32)


def reachable_mask(g: CSR, source: int) -> np.ndarray:
    """Vertices reachable from ``source`` (breadth-first search via scipy)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import breadth_first_order

    a = sp.csr_matrix((np.ones(g.m, dtype=np.int8), g.col, g.row_ptr),
                      shape=(g.n, g.n))
    order = breadth_first_order(a, int(source), directed=True,
                                return_predecessors=False)
    mask = np.zeros(g.n, dtype=bool)
    mask[order] = True
    return mask


def random_targets(g: CSR, source: int, k: int, seed: int) -> np.ndarray:
    """Up to k distinct reachable targets != source, drawn without replacement."""
    mask = reachable_mask(g, source)
    mask[source] = False
    cand = np.nonzero(mask)[0]
    rng = np.random.default_rng(seed)
    k = min(k, cand.shape[0])
    return np.sort(rng.choice(cand, size=k, replace=False)).astype(np.int32)
