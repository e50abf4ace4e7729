"""Pins for the CPU oracle: every check here is independent of the oracle's own
code (brute-force path enumeration, closed forms, a library routine, hand-built
fixtures, invariants), chosen so that a dropped term, a wrong sign or index, or
a transposed operand in the oracle fails at least one of them."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra as scipy_dijkstra

from paper_2103_12012_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64MAX = np.iinfo(np.uint64).max


def tiny_graph(seed, n=None, m=None, wmax=5, zero=True, loops=True):
    rng = np.random.default_rng(seed)
    n = n or int(rng.integers(1, 8))
    m = m if m is not None else int(rng.integers(0, 3 * n + 1))
    u = rng.integers(0, n, size=m)
    v = rng.integers(0, n, size=m)
    if not loops:
        keep = u != v
        u, v = u[keep], v[keep]
    w = rng.integers(0 if zero else 1, wmax + 1, size=u.shape[0]).astype(np.uint32)
    return gen.from_arcs(n, u, v, w)


def brute_paths(g, s):
    """Minimum over all simple s->v paths, by exhaustive DFS (pure Python)."""
    best = [None] * g.n
    best[s] = 0
    rp, col, w = g.row_ptr.tolist(), g.col.tolist(), g.w.tolist()

    def dfs(u, d, seen):
        for e in range(rp[u], rp[u + 1]):
            v = col[e]
            if v in seen:
                continue
            nd = d + int(w[e])
            if best[v] is None or nd < best[v]:
                best[v] = nd
            dfs(v, nd, seen | {v})

    dfs(s, 0, {s})
    return best


def load_golden():
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        gj = json.load(f)
    e = np.array(gj["edges_u_v_w"], dtype=np.int64)
    rp = np.zeros(gj["n"] + 1, dtype=np.int32)
    np.cumsum(np.bincount(e[:, 0], minlength=gj["n"]), out=rp[1:])
    g = gen.CSR(gj["n"], rp, e[:, 1].astype(np.int32), e[:, 2].astype(np.uint32))
    return gj, g


# ----------------------------------------------------------------- distances

@pytest.mark.parametrize("seed", range(300))
def test_dijkstra_matches_path_enumeration(orc, seed):
    g = tiny_graph(seed)
    s = seed % g.n
    d = orc.sssp(g.row_ptr, g.col, g.w, s)
    bp = brute_paths(g, s)
    for v in range(g.n):
        if bp[v] is None:
            assert d[v] == U64MAX
        else:
            assert int(d[v]) == bp[v]


@pytest.mark.parametrize("seed", range(60))
def test_dijkstra_matches_bellman_ford(orc, seed):
    g = tiny_graph(1000 + seed, n=int(8 + seed % 57), m=int(4 * (8 + seed % 57)), wmax=50)
    for s in (0, g.n // 2, g.n - 1):
        assert np.array_equal(orc.sssp(g.row_ptr, g.col, g.w, s),
                              orc.bellman_ford(g.row_ptr, g.col, g.w, s))


def test_dijkstra_matches_scipy_on_uniform(orc):
    g = gen.uniform(4096, 32768, 1)
    # scipy sums duplicate entries, so hand it the cheapest copy of each arc
    key = g.src().astype(np.int64) * g.n + g.col
    order = np.lexsort((g.w, key))
    first = np.ones(order.shape[0], bool)
    first[1:] = key[order][1:] != key[order][:-1]
    sel = order[first]
    a = sp.csr_matrix((g.w[sel].astype(np.float64), (g.src()[sel], g.col[sel])),
                      shape=(g.n, g.n))
    for s in (0, 17, 4095):
        ref = scipy_dijkstra(a, directed=True, indices=s)
        d = orc.sssp(g.row_ptr, g.col, g.w, s)
        fin = np.isfinite(ref)
        assert np.array_equal(fin, d != U64MAX)
        assert np.array_equal(ref[fin].astype(np.uint64), d[fin])


@pytest.mark.parametrize("k", [1, 7])
def test_constant_grid_closed_form(orc, k):
    g = gen.grid(23, 31, seed=0)
    g = g.with_weights(np.full(g.m, k, np.uint32))
    d = orc.sssp(g.row_ptr, g.col, g.w, 0)
    r, c = np.divmod(np.arange(g.n), 31)
    assert np.array_equal(d, (k * (r + c)).astype(np.uint64))


def test_directional_grid_closed_form(orc):
    # right arcs cost a, down arcs cost b, left/up arcs cost more than any
    # monotone path: d(r, c) = a*c + b*r from the corner.
    R, C, a, b = 17, 29, 3, 5
    g = gen.grid(R, C, seed=0)
    src = g.src()
    dcol = g.col.astype(np.int64) - src
    w = np.where(dcol == 1, a, np.where(dcol == C, b, 10**6)).astype(np.uint32)
    d = orc.sssp(g.row_ptr, g.col, w, 0)
    r, c = np.divmod(np.arange(g.n), C)
    assert np.array_equal(d, (a * c + b * r).astype(np.uint64))


def test_path_and_star(orc):
    w = np.array([3, 1, 4, 1, 5], np.uint32)
    g = gen.from_arcs(6, np.arange(5), np.arange(1, 6), w)
    d = orc.sssp(g.row_ptr, g.col, g.w, 0)
    assert d.tolist() == [0, 3, 4, 8, 9, 14]
    d = orc.sssp(g.row_ptr, g.col, g.w, 3)
    assert d[:3].tolist() == [U64MAX] * 3 and d[3:].tolist() == [0, 1, 6]
    gs = gen.from_arcs(5, np.zeros(4, int), np.arange(1, 5), np.array([9, 8, 7, 6], np.uint32))
    assert orc.sssp(gs.row_ptr, gs.col, gs.w, 0).tolist() == [0, 9, 8, 7, 6]


@pytest.mark.parametrize("seed", range(40))
def test_f32_dijkstra_equals_bellman_ford_bitwise(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 60))
    g = tiny_graph(2000 + seed, n=n, m=4 * n)
    w = rng.uniform(0.5, 1.5, size=g.m).astype(np.float32)
    d1 = orc.sssp(g.row_ptr, g.col, w, 0)
    d2 = orc.bellman_ford(g.row_ptr, g.col, w, 0)
    assert np.array_equal(d1.view(np.uint32), d2.view(np.uint32))
    # scaling by 2 is exact in binary floating point
    d3 = orc.sssp(g.row_ptr, g.col, (2 * w).astype(np.float32), 0)
    assert np.array_equal(d3, 2 * d1)


def test_f32_fold_is_left_to_right(orc):
    # 2^24 + 1 + 1: left fold in float gives 2^24 at every step (ties to even)
    g = gen.from_arcs(3, [0, 1], [1, 2])
    w = np.array([2.0**24, 1.0], np.float32)
    d = orc.sssp(g.row_ptr, g.col, w, 0)
    assert d[2] == np.float32(2.0**24)
    w2 = np.array([1.0, 2.0**24], np.float32)
    assert orc.sssp(g.row_ptr, g.col, w2, 0)[2] == np.float32(2.0**24)


# ---------------------------------------------------------- golden / pred

def test_golden_worked_example(orc):
    gj, g = load_golden()
    dist, pred, pe = orc.solve(g.row_ptr, g.col, g.w, gj["source"])
    assert dist.tolist() == gj["dist"]
    assert pe.tolist() == gj["pred_edge"]
    assert pred.tolist() == gj["pred"]
    keep = orc.trishla(g.row_ptr, g.col, g.w, method="brute")
    assert keep.tolist() == gj["trishla_keep_global"]
    assert orc.trishla(g.row_ptr, g.col, g.w).tolist() == gj["trishla_keep_global"]
    kl = orc.trishla(g.row_ptr, g.col, g.w, local_scope=True, nparts=2, method="brute")
    assert kl.tolist() == gj["trishla_keep_local_p2"]
    gvec = np.zeros(gj["n"], np.float32)
    gvec[gj["grad_targets"]] = 1
    gw = orc.grad(g.row_ptr, gj["source"], pe, gvec)
    assert gw.tolist() == gj["grad_w"]


@pytest.mark.parametrize("seed", range(200))
def test_pred_tree_paths_have_the_right_length(orc, seed):
    g = tiny_graph(3000 + seed, wmax=3, zero=False)
    s = seed % g.n
    dist, pred, pe = orc.solve(g.row_ptr, g.col, g.w, s)
    bp = brute_paths(g, s)
    src = g.src()
    for v in range(g.n):
        if bp[v] is None:
            assert pe[v] == -1 and dist[v] == 0xFFFFFFFF
            continue
        # walk the tree: the summed arc weights equal the brute-force distance
        total, x, steps = 0, v, 0
        while x != s:
            e = pe[x]
            assert e >= 0 and g.col[e] == x and src[e] == pred[x]
            total += int(g.w[e])
            x = pred[x]
            steps += 1
            assert steps <= g.n
        assert total == bp[v]
        # no arc into v with a smaller id closes at the same distance
        if v != s:
            for e in range(g.m):
                if g.col[e] == v and bp[src[e]] is not None and e < pe[v]:
                    assert bp[src[e]] + int(g.w[e]) > bp[v]


def test_zero_weight_pred_rule_can_cycle(orc):
    # With zero weights the smallest tight arc id may close a cycle: a
    # zero-weight self-loop at v is tight and can precede v's real parent.
    # Distances are unaffected; the rule is applied as stated (backward
    # therefore requires strictly positive weights).
    g = gen.from_arcs(2, [0, 1, 1], [1, 1, 1], np.array([2, 0, 5], np.uint32))
    # CSR: e0 = 0->1 (2), e1 = 1->1 (0), e2 = 1->1 (5)
    dist, pred, pe = orc.solve(g.row_ptr, g.col, g.w, 0)
    assert dist.tolist() == [0, 2] and pe.tolist() == [-1, 0]
    g = gen.from_arcs(2, [0, 0, 1], [0, 1, 1], np.array([0, 2, 0], np.uint32))
    # CSR: e0 = 0->0 (0), e1 = 0->1 (2), e2 = 1->1 (0): e1 < e2 so e1 wins
    dist, pred, pe = orc.solve(g.row_ptr, g.col, g.w, 0)
    assert dist.tolist() == [0, 2] and pe.tolist() == [-1, 1]
    g = gen.from_arcs(3, [0, 1, 2], [2, 1, 1], np.array([2, 0, 0], np.uint32))
    # CSR: e0 = 0->2 (2), e1 = 1->1 (0), e2 = 2->1 (0): 1's self-loop e1 is
    # tight and smaller than e2, so pred_edge(1) = e1 (a cycle)
    dist, pred, pe = orc.solve(g.row_ptr, g.col, g.w, 0)
    assert dist.tolist() == [0, 2, 2] and pe.tolist() == [-1, 1, 0]
    assert orc.certify(g.row_ptr, g.col, g.w, 0, dist, pe)[0] == 7


# ----------------------------------------------------------------- Trishla

def test_trishla_hand_cases(orc):
    # triangle u=0 -> y=1 -> x=2 with a direct arc 0->2
    for direct, expect in ((3, 0), (2, 1), (1, 1)):
        g = gen.from_arcs(3, [0, 0, 1], [1, 2, 2], np.array([1, direct, 1], np.uint32))
        e_direct = 1  # CSR order: 0->1, 0->2, 1->2
        for method in ("brute", "mark"):
            k = orc.trishla(g.row_ptr, g.col, g.w, method=method)
            assert k[e_direct] == expect and k[0] == 1 and k[2] == 1
    # fp32: 0.5 + 0.25 < 1 prunes, 0.5 + 0.5 = 1 keeps (strict)
    for w2, expect in ((0.25, 0), (0.5, 1)):
        g = gen.from_arcs(3, [0, 0, 1], [1, 2, 2])
        w = np.array([0.5, 1.0, w2], np.float32)
        for method in ("brute", "mark"):
            assert orc.trishla(g.row_ptr, g.col, w, method=method)[1] == expect


def test_trishla_self_loop_and_two_cycle(orc):
    # a self-loop is deleted only by a strictly cheaper 2-cycle
    g = gen.from_arcs(2, [0, 0, 1], [0, 1, 0], np.array([5, 2, 2], np.uint32))
    assert orc.trishla(g.row_ptr, g.col, g.w, method="brute").tolist() == [0, 1, 1]
    g = gen.from_arcs(2, [0, 0, 1], [0, 1, 0], np.array([4, 2, 2], np.uint32))
    assert orc.trishla(g.row_ptr, g.col, g.w, method="brute").tolist() == [1, 1, 1]
    # parallel copies never witness each other
    g = gen.from_arcs(2, [0, 0], [1, 1], np.array([1, 9], np.uint32))
    assert orc.trishla(g.row_ptr, g.col, g.w, method="mark").tolist() == [1, 1]


@pytest.mark.parametrize("L", [2, 5, 9])
def test_trishla_line_closed_forms(orc, L):
    # complete forward DAG on a line: i -> j for i < j
    u, v = zip(*[(i, j) for i in range(L) for j in range(i + 1, L)])
    u, v = np.array(u), np.array(v)
    for method in ("brute", "mark"):
        sq = orc.trishla(*_csr(L, u, v, (v - u) ** 2), method=method)
        g = gen.from_arcs(L, u, v, ((v - u) ** 2).astype(np.uint32))
        assert np.array_equal(sq.astype(bool), (g.col - g.src()) == 1)  # only i->i+1 kept
        lin = orc.trishla(*_csr(L, u, v, v - u), method=method)
        assert lin.all()  # every detour ties: nothing deleted


def _csr(n, u, v, w):
    g = gen.from_arcs(n, u, v, np.asarray(w, dtype=np.uint32))
    return g.row_ptr, g.col, g.w


def test_trishla_grid_deletes_nothing(orc):
    g = gen.grid(40, 50, seed=3)  # bipartite: no directed triangle exists
    assert orc.trishla(g.row_ptr, g.col, g.w).all()
    assert orc.trishla(g.row_ptr, g.col, g.w, method="brute").all()


@pytest.mark.parametrize("seed", range(150))
def test_trishla_brute_equals_mark_and_scopes(orc, seed):
    g = tiny_graph(4000 + seed, wmax=6)
    kb = orc.trishla(g.row_ptr, g.col, g.w, method="brute")
    km = orc.trishla(g.row_ptr, g.col, g.w, method="mark")
    assert np.array_equal(kb, km)
    P = 1 + seed % 4
    lb = orc.trishla(g.row_ptr, g.col, g.w, True, P, method="brute")
    lm = orc.trishla(g.row_ptr, g.col, g.w, True, P, method="mark")
    assert np.array_equal(lb, lm)
    assert np.all(lb >= kb)  # LOCAL deletes a subset of GLOBAL
    assert np.array_equal(orc.trishla(g.row_ptr, g.col, g.w, True, 1, method="mark"), km)


@pytest.mark.parametrize("seed", range(120))
def test_trishla_preserves_every_distance(orc, seed):
    # pruning safety: distances from every source are unchanged, checked by
    # brute-force path enumeration on both graphs
    g = tiny_graph(5000 + seed, wmax=5)
    keep = orc.trishla(g.row_ptr, g.col, g.w).astype(bool)
    src = g.src()
    gp = gen.from_arcs(g.n, src[keep], g.col[keep], g.w[keep])
    for s in range(g.n):
        assert brute_paths(g, s) == brute_paths(gp, s)


def test_trishla_pruned_arcs_have_a_witness_and_kept_arcs_none(orc):
    rng = np.random.default_rng(7)
    for t in range(30):
        g = tiny_graph(6000 + t, n=12, m=60, wmax=9)
        keep = orc.trishla(g.row_ptr, g.col, g.w)
        arcs = {}
        for e, (a, b) in enumerate(zip(g.src(), g.col)):
            arcs.setdefault((int(a), int(b)), []).append(int(g.w[e]))
        for e, (a, b) in enumerate(zip(g.src(), g.col)):
            a, b = int(a), int(b)
            cheapest = min((min(arcs[(a, y)]) + min(arcs[(y, b)])
                            for y in range(g.n) if y not in (a, b)
                            and (a, y) in arcs and (y, b) in arcs), default=None)
            has = cheapest is not None and cheapest < int(g.w[e])
            assert bool(keep[e]) == (not has)


def test_trishla_f32_brute_equals_mark(orc):
    for t in range(40):
        g = tiny_graph(7000 + t, n=10, m=40)
        rng = np.random.default_rng(t)
        w = rng.choice(np.array([0.25, 0.5, 0.75, 1.0, 1.25], np.float32), size=g.m)
        assert np.array_equal(orc.trishla(g.row_ptr, g.col, w, method="brute"),
                              orc.trishla(g.row_ptr, g.col, w, method="mark"))


# ------------------------------------------------------------- certificate

def test_certificate_accepts_oracle_and_rejects_mutations(orc):
    g = gen.uniform(300, 1500, 11)
    dist, pred, pe = orc.solve(g.row_ptr, g.col, g.w, 0)
    assert orc.certify(g.row_ptr, g.col, g.w, 0, dist, pe) == (0, -1)
    reached = np.nonzero((dist != 0xFFFFFFFF) & (np.arange(g.n) != 0))[0]
    v = int(reached[len(reached) // 2])
    bad = dist.copy(); bad[v] -= 1
    assert orc.certify(g.row_ptr, g.col, g.w, 0, bad, pe)[0] != 0
    bad = dist.copy(); bad[v] += 1
    assert orc.certify(g.row_ptr, g.col, g.w, 0, bad, pe)[0] != 0
    bad = dist.copy(); bad[v] = 0xFFFFFFFF
    assert orc.certify(g.row_ptr, g.col, g.w, 0, bad, pe)[0] != 0
    bp = pe.copy(); bp[v] = (bp[v] + 1) % g.m
    assert orc.certify(g.row_ptr, g.col, g.w, 0, dist, bp)[0] != 0
    bp = pe.copy(); bp[v] = -1
    assert orc.certify(g.row_ptr, g.col, g.w, 0, dist, bp)[0] != 0
    bad = dist.copy(); bad[0] = 1
    assert orc.certify(g.row_ptr, g.col, g.w, 0, bad, pe)[0] == 1
    # a larger tight edge than the minimum is rejected
    src = g.src()
    for x in reached:
        tight = [e for e in range(g.m) if g.col[e] == x and dist[src[e]] != 0xFFFFFFFF
                 and int(dist[src[e]]) + int(g.w[e]) == int(dist[x])]
        if len(tight) > 1:
            bp = pe.copy(); bp[x] = tight[-1]
            assert orc.certify(g.row_ptr, g.col, g.w, 0, dist, bp)[0] == 6
            break
    else:
        pytest.fail("no vertex with two tight in-arcs in this instance")


def test_certificate_rejects_cycle(orc):
    # zero-weight 2-cycle 1<->2 below the true parents: pointing the preds at
    # each other is tight and feasible but never reaches the source
    g = gen.from_arcs(3, [0, 0, 1, 2], [1, 2, 2, 1], np.array([1, 1, 0, 0], np.uint32))
    dist = np.array([0, 1, 1], np.uint32)
    pe = np.array([-1, 3, 2], np.int32)
    assert orc.certify(g.row_ptr, g.col, g.w, 0, dist, pe)[0] in (6, 7)


# ---------------------------------------------------------------- gradient

def test_grad_euler_identity(orc):
    # L = sum_t d(t) is 1-homogeneous in w: <dL/dw, w> = L (exact for ints)
    g = gen.rmat(10, 10, weight="u32", whi=20)
    s = int(np.argmax(g.out_degree()))
    dist, pred, pe = orc.solve(g.row_ptr, g.col, g.w, s)
    rng = np.random.default_rng(0)
    cand = np.nonzero(dist != 0xFFFFFFFF)[0]
    t = rng.choice(cand, size=min(200, len(cand)), replace=False)
    gv = np.zeros(g.n, np.float32)
    gv[t] = rng.integers(1, 4, size=t.shape[0])
    gw = orc.grad(g.row_ptr, s, pe, gv)
    L = float(np.dot(gv.astype(np.float64), dist.astype(np.float64)))
    assert float(np.dot(gw.astype(np.float64), g.w.astype(np.float64))) == L


def test_grad_matches_finite_differences(orc):
    g = gen.rmat(7, 70, weight="f32", wlo=0.5, whi=1.5)
    s = int(np.argmax(g.out_degree()))
    d = orc.sssp(g.row_ptr, g.col, g.w.astype(np.float64), s)
    pe, _ = orc.pred(g.row_ptr, g.col, g.w.astype(np.float64), s, d)
    gv = np.zeros(g.n, np.float32)
    tg = np.nonzero(np.isfinite(d))[0][::3]
    gv[tg] = 1.0
    gw = orc.grad(g.row_ptr, s, pe, gv)
    fd, valid = orc.finite_diff(g.row_ptr, g.col, g.w, s, gv, eps=1e-4)
    assert valid.mean() > 0.95
    np.testing.assert_allclose(fd[valid], gw[valid], atol=1e-6, rtol=1e-6)
    assert np.abs(gw).sum() > 0


# ----------------------------------------------- floating-point pins (fp32 / f64)
#
# The fp32 path sums costs left to right from the source in float32 (a
# rounding step per arc), and its predecessor rule compares in float32.  The
# brute force below enumerates simple paths in pure Python and folds each
# path's costs in the requested numpy dtype, one rounding per arc; with
# positive costs the least fold over simple paths equals the least over all
# walks (a cycle never lowers a fold), which is the shortest-path value.

def brute_paths_fp(g, w, s, dtype):
    """Least left-fold (in ``dtype``) over all simple s->v paths, or None."""
    best = [None] * g.n
    best[s] = dtype(0)
    rp, col = g.row_ptr.tolist(), g.col.tolist()
    wl = [dtype(x) for x in w]

    def dfs(u, d, seen):
        for e in range(rp[u], rp[u + 1]):
            v = col[e]
            if v in seen:
                continue
            nd = dtype(d + wl[e])
            if best[v] is None or nd < best[v]:
                best[v] = nd
            dfs(v, nd, seen | {v})

    dfs(s, dtype(0), {s})
    return best


def check_fp_pred(g, w, s, dist, pe, dtype, bp):
    """Every reached v != s has a tight predecessor arc in ``dtype``
    arithmetic (tail's brute distance + cost == v's brute distance), its
    tree path folds to the brute distance, and no smaller arc id into v is
    tight; unreached vertices have none."""
    src = g.src()
    wl = [dtype(x) for x in w]
    for v in range(g.n):
        if bp[v] is None:
            assert pe[v] == -1 and np.isinf(dist[v])
            continue
        assert dist[v] == bp[v]
        if v == s:
            assert pe[v] == -1
            continue
        e = int(pe[v])
        assert e >= 0 and g.col[e] == v, (v, e)
        u = int(src[e])
        assert bp[u] is not None and dtype(bp[u] + wl[e]) == bp[v]
        for e2 in range(g.m):
            if g.col[e2] == v and e2 < e and bp[int(src[e2])] is not None:
                assert dtype(bp[int(src[e2])] + wl[e2]) > bp[v], (v, e2, e)
        # walk the tree back to s, then fold forward in dtype
        path, x = [], v
        while x != s:
            path.append(int(pe[x]))
            x = int(src[pe[x]])
            assert len(path) <= g.n
        acc = dtype(0)
        for a in reversed(path):
            acc = dtype(acc + wl[a])
        assert acc == bp[v]


@pytest.mark.parametrize("seed", range(120))
def test_pred_f32_ties_against_path_enumeration(orc, seed):
    # costs from {0.25, 0.5, 0.75}: sums are exact and ties are frequent, so
    # the smallest-id rule among several tight arcs is exercised
    g = tiny_graph(8000 + seed, n=int(2 + seed % 7), m=int(3 * (2 + seed % 7)), zero=False)
    rng = np.random.default_rng(seed)
    w = rng.choice(np.array([0.25, 0.5, 0.75], np.float32), size=g.m)
    s = seed % g.n
    dist, pred, pe = orc.solve(g.row_ptr, g.col, w, s)
    check_fp_pred(g, w, s, dist, pe, np.float32, brute_paths_fp(g, w, s, np.float32))
    src = g.src()
    assert np.array_equal(pred[pe >= 0], src[pe[pe >= 0]])
    assert np.all(pred[pe < 0] == -1)


@pytest.mark.parametrize("seed", range(120))
def test_pred_f32_rounding_against_path_enumeration(orc, seed):
    # costs whose sums round in float32 (a distance offset of 2^20 in front
    # of the tiny graph makes almost every sum inexact): a tight arc is
    # decided in float32, so a predecessor test made in double finds no
    # tight arc for most vertices and fails here
    rng = np.random.default_rng(100 + seed)
    n = int(3 + seed % 6)
    g0 = tiny_graph(9000 + seed, n=n, m=4 * n, zero=False)
    # vertex n is a new source joined to every vertex by an arc of cost
    # ~2^20, so every distance is large and its sums round
    u = np.concatenate([g0.src(), np.full(n, n)])
    v = np.concatenate([g0.col, np.arange(n)])
    w0 = rng.uniform(0.1, 10.0, size=g0.m).astype(np.float32)
    big = (2.0**20 + rng.uniform(0, 64, size=n)).astype(np.float32)
    g = gen.from_arcs(n + 1, u, v, np.concatenate([w0, big]).astype(np.float32))
    w = g.w
    s = n
    dist, pred, pe = orc.solve(g.row_ptr, g.col, w, s)
    check_fp_pred(g, w, s, dist, pe, np.float32, brute_paths_fp(g, w, s, np.float32))


@pytest.mark.parametrize("seed", range(60))
def test_sssp_and_pred_f64_against_path_enumeration(orc, seed):
    rng = np.random.default_rng(300 + seed)
    g = tiny_graph(9500 + seed, n=int(2 + seed % 7), m=int(4 * (2 + seed % 7)), zero=False)
    # half the cases with exact ties (multiples of 1/4), half with rounding
    if seed % 2:
        w = rng.choice(np.array([0.25, 0.5, 0.75, 1.0]), size=g.m).astype(np.float64)
    else:
        w = (1e15 * rng.uniform(0.5, 1.5, size=g.m)).astype(np.float64) / 3.0
    s = seed % g.n
    d = orc.sssp(g.row_ptr, g.col, w, s)
    pe, pv = orc.pred(g.row_ptr, g.col, w, s, d)
    check_fp_pred(g, w, s, d, pe, np.float64, brute_paths_fp(g, w, s, np.float64))


def test_sssp_f64_matches_scipy(orc):
    # a library Dijkstra in float64: same left fold, so bit-identical
    g = gen.rmat(12, 12, weight="f32", wlo=0.5, whi=1.5)
    w = g.w.astype(np.float64) * (1.0 + 1.0 / 3.0)  # sums that round in float64
    a = sp.csr_matrix((w, g.col, g.row_ptr), shape=(g.n, g.n))
    for s in gen.random_sources(g, 3, 12):
        ref = scipy_dijkstra(a, directed=True, indices=int(s))
        d = orc.sssp(g.row_ptr, g.col, w, int(s))
        assert np.array_equal(np.isfinite(ref), np.isfinite(d))
        fin = np.isfinite(ref)
        assert np.array_equal(ref[fin].view(np.uint64), d[fin].view(np.uint64))


def test_certificate_f32_rejects_mutations(orc):
    g = gen.rmat(9, 9)
    rng = np.random.default_rng(9)
    w = rng.choice(np.array([0.25, 0.5, 0.75, 1.0], np.float32), size=g.m)
    s = int(np.argmax(g.out_degree()))
    dist, pred, pe = orc.solve(g.row_ptr, g.col, w, s)
    assert orc.certify(g.row_ptr, g.col, w, s, dist, pe) == (0, -1)
    reached = np.nonzero(np.isfinite(dist) & (np.arange(g.n) != s))[0]
    v = int(reached[len(reached) // 2])
    up = np.float32(np.inf)
    for bad_v in (np.nextafter(dist[v], np.float32(0)), np.nextafter(dist[v], up), up):
        bad = dist.copy()
        bad[v] = bad_v
        assert orc.certify(g.row_ptr, g.col, w, s, bad, pe)[0] != 0
    bad = dist.copy()
    bad[s] = np.float32(0.25)
    assert orc.certify(g.row_ptr, g.col, w, s, bad, pe)[0] == 1
    bp = pe.copy(); bp[v] = (bp[v] + 1) % g.m
    assert orc.certify(g.row_ptr, g.col, w, s, dist, bp)[0] != 0
    bp = pe.copy(); bp[v] = -1
    assert orc.certify(g.row_ptr, g.col, w, s, dist, bp)[0] == 4
    # an unreached vertex given a predecessor
    unreached = np.nonzero(~np.isfinite(dist))[0]
    if unreached.size:
        bp = pe.copy(); bp[int(unreached[0])] = 0
        assert orc.certify(g.row_ptr, g.col, w, s, dist, bp)[0] == 3
    # a larger tight arc than the smallest one
    src = g.src()
    tight = np.isfinite(dist[src]) & ((dist[src] + w).astype(np.float32) == dist[g.col])
    tight &= g.col != s
    cnt = np.bincount(g.col[tight], minlength=g.n)
    x = int(np.nonzero(cnt > 1)[0][0])
    last = int(np.nonzero(tight & (g.col == x))[0][-1])
    bp = pe.copy(); bp[x] = last
    assert orc.certify(g.row_ptr, g.col, w, s, dist, bp)[0] == 6
    # a cycle of zero-cost arcs below the true parents
    gc = gen.from_arcs(3, [0, 0, 1, 2], [1, 2, 2, 1])
    wc = np.array([1, 1, 0, 0], np.float32)
    assert orc.certify(gc.row_ptr, gc.col, wc, 0, np.array([0, 1, 1], np.float32),
                       np.array([-1, 3, 2], np.int32))[0] in (6, 7)
    assert orc.certify(gc.row_ptr, gc.col, wc, 0, np.array([0, 1, 1], np.float32),
                       np.array([-1, 0, 1], np.int32)) == (0, -1)


# Trishla with fp32 costs compares w1 + w2 < W exactly (real numbers).  The
# cases below need more than float32 (the float sum rounds) or more than the
# double sum (the exponents are more than 29 bits apart, so the double sum
# rounds too and the exact remainder decides).

F32_EDGE_COSTS = np.array([
    1.0, 2.0**-60, 2.0**-61, 1.0 + 2.0**-23, 1.0 + 2.0**-22, 2.0**-24 + 2.0**-30,
    2.0**-24, 2.0**-23, 0.5, 0.5 + 2.0**-24, 3.0, 2.0, 1.5,
], np.float32)


def trishla_exact(g, w):
    """Keep mask from exact rational arithmetic (pure Python)."""
    from fractions import Fraction

    src = g.src().tolist()
    col = g.col.tolist()
    fw = [Fraction(float(x)) for x in w]
    arcs = {}
    for e in range(g.m):
        arcs.setdefault((src[e], col[e]), []).append(fw[e])
    keep = np.ones(g.m, np.uint8)
    for e in range(g.m):
        a, b = src[e], col[e]
        for y in range(g.n):
            if y in (a, b) or (a, y) not in arcs or (y, b) not in arcs:
                continue
            if min(arcs[(a, y)]) + min(arcs[(y, b)]) < fw[e]:
                keep[e] = 0
                break
    return keep


def test_trishla_f32_inexact_sums_hand_cases(orc):
    g = gen.from_arcs(3, [0, 0, 1], [1, 2, 2])  # e0 = 0->1, e1 = 0->2, e2 = 1->2
    one_up = np.nextafter(np.float32(1), np.float32(2))
    cases = [
        # (w(0->1), w(0->2), w(1->2), keep of 0->2)
        (1.0, 1.0, 2.0**-60, 1),     # 1 + 2^-60 > 1: the double sum rounds to 1
        (1.0, one_up, 2.0**-60, 0),  # 1 + 2^-60 < 1 + 2^-23
        (2.0**-60, 1.0, 1.0, 1),     # operands swapped
        (2.0**-61, 2.0**-60, 2.0**-61, 1),  # exact tie: strict comparison keeps
        (1.0, one_up, 2.0**-24 + 2.0**-30, 0),  # float32 sum rounds up to W
        (1.0, 1.0 + 2.0**-22, 2.0**-23 + 2.0**-24, 0),
        (1.0, one_up, 2.0**-23, 1),  # exact tie at the ulp
    ]
    for w1, W, w2, expect in cases:
        w = np.array([w1, W, w2], np.float32)
        ref = trishla_exact(g, w)
        assert ref[1] == expect, (w1, W, w2)
        for method in ("brute", "mark"):
            assert orc.trishla(g.row_ptr, g.col, w, method=method).tolist() == ref.tolist(), \
                (method, w1, W, w2)


@pytest.mark.parametrize("seed", range(80))
def test_trishla_f32_matches_exact_arithmetic(orc, seed):
    g = tiny_graph(11000 + seed, n=int(3 + seed % 8), m=int(5 * (3 + seed % 8)), loops=False)
    rng = np.random.default_rng(seed)
    w = rng.choice(F32_EDGE_COSTS, size=g.m)
    ref = trishla_exact(g, w)
    for method in ("brute", "mark"):
        assert np.array_equal(orc.trishla(g.row_ptr, g.col, w, method=method), ref), method


# ------------------------------------------------------------------ overflow

def test_overflow_decided_by_final_distances(orc):
    # a path whose sum does not fit is no error while a shorter one exists
    g = gen.from_arcs(3, [0, 0, 2], [1, 2, 1], np.array([1, 0xFFFFFFF0, 0x100], np.uint32))
    dist, pred, pe = orc.solve(g.row_ptr, g.col, g.w, 0)
    assert dist.tolist() == [0, 1, 0xFFFFFFF0] and pe.tolist() == [-1, 0, 1]
    g = gen.from_arcs(2, [0, 1], [1, 0], np.array([0xFFFFFFF0, 0x100], np.uint32))
    assert orc.solve(g.row_ptr, g.col, g.w, 0)[0].tolist() == [0, 0xFFFFFFF0]
    # the largest representable distance fits; one more does not
    g = gen.from_arcs(2, [0], [1], np.array([0xFFFFFFFE], np.uint32))
    assert orc.solve(g.row_ptr, g.col, g.w, 0)[0].tolist() == [0, 0xFFFFFFFE]
    g = gen.from_arcs(3, [0, 1], [1, 2], np.array([0xFFFFFFFE, 1], np.uint32))
    with pytest.raises(OverflowError):
        orc.solve(g.row_ptr, g.col, g.w, 0)
    g = gen.from_arcs(3, [0, 1], [1, 2], np.array([0xF0000000, 0x20000000], np.uint32))
    with pytest.raises(OverflowError):
        orc.solve(g.row_ptr, g.col, g.w, 0)


def test_overflow_f32(orc):
    big = np.float32(3e38)
    g = gen.from_arcs(3, [0, 0, 2], [1, 2, 1])
    dist, _, pe = orc.solve(g.row_ptr, g.col, np.array([1.0, big, big], np.float32), 0)
    assert dist.tolist() == [0.0, 1.0, float(big)] and pe.tolist() == [-1, 0, 1]
    g = gen.from_arcs(4, [0, 1], [1, 2])  # vertex 3 is unreachable: no error
    with pytest.raises(OverflowError):
        orc.solve(g.row_ptr, g.col, np.array([big, big], np.float32), 0)
    dist, _, _ = orc.solve(g.row_ptr, g.col, np.array([1.0, 2.0], np.float32), 0)
    assert dist.tolist() == [0.0, 1.0, 3.0, float("inf")]
