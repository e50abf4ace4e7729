"""GPU parity of sssp_solve against the oracle: bit-exact distances,
predecessors and predecessor edges, over tiny graphs with zero weights,
multi-edges and self-loops, the small uniform configuration under sweeps of
delta / partitions / workgroup shape, R-MAT and grid graphs up to the full
benchmark sizes."""
import numpy as np
import pytest

import oracle
from paper_2103_12012_amd import gen
from helpers import assert_solve_parity, dev, gpu_solve, sssp_mod, tiny_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    g = gen.uniform(4096, 32768, seed=1)
    return g, dev(g), oracle.solve(g.row_ptr, g.col, g.w, 0)


def test_golden_worked_example():
    import json, os
    with open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")) as f:
        gj = json.load(f)
    e = np.array(gj["edges_u_v_w"])
    g = gen.from_arcs(gj["n"], e[:, 0], e[:, 1], e[:, 2].astype(np.uint32))
    for P in (1, 2, 7):
        dist, pred, pe = gpu_solve(g, gj["source"], num_partitions=P)
        assert dist.tolist() == gj["dist"]
        assert pe.tolist() == gj["pred_edge"]
        assert pred.tolist() == gj["pred"]


@pytest.mark.parametrize("seed", range(40))
def test_tiny_graphs(seed):
    g = tiny_graph(seed)
    s = seed % g.n
    P = 1 + seed % 9
    delta = [1, 3, 0, -1][seed % 4]
    assert_solve_parity(g, s, gpu_solve(g, s, num_partitions=P, delta=delta))


def test_c1_default(c1):
    g, d, ref = c1
    assert_solve_parity(g, 0, gpu_solve(g, 0, d=d, num_partitions=4), ref)


@pytest.mark.parametrize("delta", [1, 100, 400, -1])
@pytest.mark.parametrize("P", [1, 2, 4, 7, 256, 4096])
def test_c1_delta_partition_sweep(c1, delta, P):
    g, d, ref = c1
    assert_solve_parity(g, 0, gpu_solve(g, 0, d=d, num_partitions=P, delta=delta), ref)


@pytest.mark.parametrize("wg", [256, 512, 1024])
@pytest.mark.parametrize("grid", [1, 7, 0])
def test_c1_workgroup_sweep(c1, wg, grid):
    g, d, ref = c1
    assert_solve_parity(g, 0, gpu_solve(g, 0, d=d, num_partitions=4, wg_size=wg,
                                        num_workgroups=grid), ref)


def test_c1_deterministic_repeats(c1):
    g, d, ref = c1
    s = sssp_mod().Solver(*d, num_partitions=4)
    first = None
    for _ in range(10):
        dist, pred, pe = s(0, sync=True)
        cur = (dist.cpu().numpy().copy(), pe.cpu().numpy().copy())
        if first is None:
            first = cur
        assert np.array_equal(cur[0], first[0]) and np.array_equal(cur[1], first[1])


@pytest.mark.parametrize("scale,seed", [(10, 1), (12, 2), (14, 3), (16, 4)])
def test_rmat_sources(scale, seed):
    g = gen.rmat(scale, seed)
    d = dev(g)
    for s in gen.random_sources(g, 3, seed):
        assert_solve_parity(g, s, gpu_solve(g, s, d=d))


def test_rmat_fp32():
    g = gen.rmat(14, 22, weight="f32", wlo=0.5, whi=1.5)
    s = int(gen.random_sources(g, 1, 5)[0])
    assert_solve_parity(g, s, gpu_solve(g, s))


@pytest.mark.parametrize("R,C", [(1, 1), (1, 300), (300, 1), (97, 131)])
def test_grid_small(R, C):
    g = gen.grid(R, C, seed=3)
    assert_solve_parity(g, 0, gpu_solve(g, 0, num_partitions=max(1, g.n // 512)))


@pytest.mark.parametrize("opts", [dict(), dict(delta=1, num_partitions=7),
                                  dict(delta=-1, num_partitions=64), dict(buffer_cross=True),
                                  dict(local_heap=True)])
def test_rmat_mostly_zero_costs(opts):
    """R-MAT 14 with costs in {0, 1, 2}: long zero-cost paths and zero-cost
    cycles, so most labels tie and the predecessor rule (the smallest arc id
    among tight arcs) decides; bit-exact against the oracle in every mode."""
    g0 = gen.rmat(14, 61)
    w = np.random.default_rng(61).choice(np.array([0, 0, 0, 1, 2], np.uint32), size=g0.m)
    g = gen.CSR(g0.n, g0.row_ptr, g0.col, w)
    s = int(gen.random_sources(g, 1, 61)[0])
    assert_solve_parity(g, s, gpu_solve(g, s, **opts))


def test_isolated_source_and_empty_graph():
    g = gen.from_arcs(5, [], [], np.zeros(0, np.uint32))
    dist, pred, pe = gpu_solve(g, 3)
    assert dist.tolist() == [0xFFFFFFFF] * 3 + [0, 0xFFFFFFFF]
    assert pe.tolist() == [-1] * 5 and pred.tolist() == [-1] * 5
    g = gen.from_arcs(1, [], [], np.zeros(0, np.uint32))
    assert gpu_solve(g, 0)[0].tolist() == [0]


def test_max_rounds_gives_upper_bounds_and_warm_restartable():
    g = gen.rmat(14, 8)
    s = int(gen.random_sources(g, 1, 8)[0])
    rp, c, w = dev(g)
    S = sssp_mod()
    solver = S.Solver(rp, c, w, max_rounds=2, num_partitions=64, stats=True)
    with pytest.raises(S.SSSPError) as ei:
        solver(s, sync=True)
    assert ei.value.code == -8
    dist = solver.dist.cpu().numpy().view(np.uint32)
    dr, _, _ = oracle.solve(g.row_ptr, g.col, g.w, s)
    fin = dist != 0xFFFFFFFF
    assert np.all(dist[fin] >= dr[fin])  # every finite label is a real path
    assert fin.sum() < (dr != 0xFFFFFFFF).sum() or not np.array_equal(dist, dr)


def test_stats_counters(c1):
    g, d, ref = c1
    S = sssp_mod()
    solver = S.Solver(*d, num_partitions=4, stats=True)
    solver(0, sync=True)
    st = solver.stats.read()
    assert st["status"] == 0 and st["num_partitions"] == 4
    reached_edges = int(g.out_degree()[ref[0] != 0xFFFFFFFF].sum())
    assert st["edges_relaxed"] >= reached_edges
    assert st["vertices_expanded"] >= int((ref[0] != 0xFFFFFFFF).sum())
    assert 0 < st["label_updates"] <= st["edges_relaxed"]
    assert st["cross_updates"] <= st["label_updates"]


def test_rmat20_full_size_prune_then_solve():
    """The benchmark workload at full size: R-MAT scale 20, pruned, solved
    from a random non-isolated source with 256 partitions."""
    g = gen.rmat(20, 20)
    s = int(gen.random_sources(g, 1, 20)[0])
    S = sssp_mod()
    rp, c, w = dev(g)
    keep, (prp, pc, pw, emap) = S.prune(rp, c, w, num_partitions=256)
    dist, pred, pe = S.solve(prp, pc, pw, s, num_partitions=256)
    dist = dist.cpu().numpy().view(np.uint32)
    pe = pe.cpu().numpy()
    emap = emap.cpu().numpy()
    pe_orig = np.where(pe >= 0, emap[np.maximum(pe, 0)], -1)
    assert_solve_parity(g, s, (dist, pred.cpu().numpy(), pe_orig))
    assert oracle.certify(g.row_ptr, g.col, g.w, s, dist, pe_orig) == (0, -1)


@pytest.mark.parametrize("opts", [dict(num_partitions=512, delta=4000, lag=2), dict()])
def test_grid4096_full_size(opts):
    """Road-like grid at full size (16.8M vertices, 67M arcs) from a corner,
    with the tuned and with the default options: checked with the LP-dual
    certificate (exact distances and the smallest-tight-edge predecessor)
    and against the oracle."""
    g = gen.grid(4096, 4096, seed=3)
    dist, pred, pe = gpu_solve(g, 0, **opts)
    assert oracle.certify(g.row_ptr, g.col, g.w, 0, dist, pe) == (0, -1)
    assert_solve_parity(g, 0, (dist, pred, pe))


def _auto_width(g, factor):
    """Expected automatic bucket width: factor x the mean of the sampled
    costs (4096 arcs at a fixed stride), rounded up for integer costs."""
    m = g.m
    k = min(m, 4096)
    idx = (np.arange(k, dtype=np.int64) * m) // k
    mean = g.w[idx].astype(np.float64).mean()
    return int(np.ceil(factor * mean))


@pytest.mark.parametrize("kind", ["dense", "sparse"])
def test_auto_delta_width_and_parity(kind):
    """Automatic options (no cache entry): the device picks the bucket width
    from sampled costs (0.5x the mean at average degree >= 8, 16x below) and
    the result still equals the oracle."""
    g = gen.rmat(11, 41) if kind == "dense" else gen.grid(96, 80, seed=9)
    factor = 0.5 if g.m >= 8 * g.n else 16.0
    S = sssp_mod()
    rp, c, w = dev(g)
    solver = S.Solver(rp, c, w, no_autotune=True, stats=True)
    s = 0 if kind == "sparse" else int(gen.random_sources(g, 1, 41)[0])
    dist, pred, pe = solver(s, sync=True)
    st = solver.stats.read()
    assert st["delta_bits"] == _auto_width(g, factor)
    assert_solve_parity(g, s, (dist.cpu().numpy().view(np.uint32), pred.cpu().numpy(),
                               pe.cpu().numpy()))


def test_auto_delta_fp32():
    g = gen.rmat(10, 42, weight="f32", wlo=0.5, whi=1.5)
    S = sssp_mod()
    rp, c, w = dev(g)
    solver = S.Solver(rp, c, w, no_autotune=True, stats=True)
    s = int(gen.random_sources(g, 1, 42)[0])
    dist, pred, pe = solver(s, sync=True)
    st = solver.stats.read()
    k = min(g.m, 4096)
    idx = (np.arange(k, dtype=np.int64) * g.m) // k
    width = np.float32(0.5 * g.w[idx].astype(np.float64).mean())
    assert abs(np.uint32(st["delta_bits"]).view(np.float32) - width) <= 1e-6 * width
    assert_solve_parity(g, s, (dist.cpu().numpy(), pred.cpu().numpy(), pe.cpu().numpy()))


@pytest.mark.parametrize("delta", [-1.0, 1.0])
def test_long_path_in_one_partition(delta):
    """A 3000-vertex directed path inside one partition: one frontier vertex
    per round, so a batch reaches its round cap and hands its queue back to
    the inbox; the result must still be exact."""
    n = 3000
    u = np.arange(n - 1)
    w = np.random.default_rng(3).integers(1, 9, size=n - 1).astype(np.uint32)
    g = gen.from_arcs(n, u, u + 1, w)
    assert_solve_parity(g, 0, gpu_solve(g, 0, num_partitions=1, delta=delta, lag=-1))


def test_hub_floods_frontier_capacity():
    """A hub with 40000 out-arcs inside one 32768-vertex partition fills far
    more than one LDS frontier of inbox entries at once (the truncated
    gather path), plus a second layer of arcs among the leaves."""
    n = 40001
    rng = np.random.default_rng(5)
    u = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(1, n, size=60000)])
    v = np.concatenate([np.arange(1, n), rng.integers(1, n, size=60000)])
    w = rng.integers(1, 50, size=u.size).astype(np.uint32)
    keep = u != v
    g = gen.from_arcs(n, u[keep], v[keep], w[keep])
    for P in (2, 64):
        assert_solve_parity(g, 0, gpu_solve(g, 0, num_partitions=P, delta=1000.0))


def test_largest_partition_block():
    """P = 1 on a graph of 140000 vertices is raised so that no block exceeds
    65536 vertices (the LDS dedupe bitmap and gather mask of a partition);
    blocks of exactly 65536 vertices (P = 2 on 131072) fill both, and blocks
    of 65535 (P = 2 on 131069) put the second block's 65535 vertices over
    2049 inbox words; the results are exact."""
    S = sssp_mod()
    for n, P, want in ((140000, 1, 3), (131072, 2, 2), (131069, 2, 2)):
        g = gen.uniform(n, 4 * n, seed=8)
        rp, c, w = dev(g)
        solver = S.Solver(rp, c, w, num_partitions=P, stats=True)
        dist, pred, pe = solver(0, sync=True)
        assert solver.stats.read()["num_partitions"] == want
        assert_solve_parity(g, 0, (dist.cpu().numpy().view(np.uint32), pred.cpu().numpy(),
                                   pe.cpu().numpy()))


def test_hub_wakes_more_units_than_the_wakeup_table():
    """A hub with arcs into 20000 single-vertex partitions: one batch pushes
    into far more units than the LDS table that gathers the wakeups holds
    (512 slots), so most wakeups take the direct path; a second layer of
    arcs among the leaves keeps several rounds of cross-partition pushes
    going.  Exact against the oracle, and with several workgroup shapes."""
    n = 20001
    rng = np.random.default_rng(6)
    u = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(1, n, size=40000)])
    v = np.concatenate([np.arange(1, n), rng.integers(1, n, size=40000)])
    w = rng.integers(1, 30, size=u.size).astype(np.uint32)
    keep = u != v
    g = gen.from_arcs(n, u[keep], v[keep], w[keep])
    ref = oracle.solve(g.row_ptr, g.col, g.w, 0)
    for kw in (dict(num_partitions=n), dict(num_partitions=n, wg_size=256, lag=-1),
               dict(num_partitions=4000, delta=-1.0)):
        assert_solve_parity(g, 0, gpu_solve(g, 0, **kw), ref)
