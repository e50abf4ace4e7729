"""GPU parity of the solve's optional modes against the oracle, through the
C ABI: buffered cross-partition updates (SSSP_F_BUFFER_CROSS) and the
literal local rule of Alg. 3, one vertex at a time from an LDS binary heap
(SSSP_F_LOCAL_HEAP).  Every mode must give the oracle's distances,
predecessors and predecessor arcs bit for bit, whatever delta, partition
count, workgroup shape or schedule."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_12012_amd import gen
from helpers import assert_solve_parity, dev, gpu_solve, sssp_mod, tiny_graph

pytestmark = pytest.mark.gpu

MODES = {
    "buffered": dict(buffer_cross=True),
    "heap": dict(local_heap=True),
}


@pytest.fixture(scope="module")
def c1():
    g = gen.uniform(4096, 32768, seed=1)
    return g, dev(g), oracle.solve(g.row_ptr, g.col, g.w, 0)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(24))
def test_tiny_graphs(mode, seed):
    g = tiny_graph(100 + seed)
    s = seed % g.n
    P = 1 + seed % 9
    delta = [1, 3, 0, -1][seed % 4]
    assert_solve_parity(g, s, gpu_solve(g, s, num_partitions=P, delta=delta, **MODES[mode]))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("delta", [1, 100, 400, -1])
@pytest.mark.parametrize("P", [1, 4, 7, 256, 4096])
def test_c1_delta_partition_sweep(c1, mode, delta, P):
    g, d, ref = c1
    assert_solve_parity(g, 0, gpu_solve(g, 0, d=d, num_partitions=P, delta=delta,
                                        **MODES[mode]), ref)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("wg", [256, 512, 1024])
@pytest.mark.parametrize("grid", [1, 7, 0])
def test_c1_workgroup_sweep(c1, mode, wg, grid):
    g, d, ref = c1
    assert_solve_parity(g, 0, gpu_solve(g, 0, d=d, num_partitions=64, wg_size=wg,
                                        num_workgroups=grid, **MODES[mode]), ref)


@pytest.mark.parametrize("mode", MODES)
def test_rmat_and_fp32(mode):
    for scale, seed in ((12, 2), (16, 4)):
        g = gen.rmat(scale, seed)
        d = dev(g)
        for s in gen.random_sources(g, 2, seed):
            assert_solve_parity(g, s, gpu_solve(g, s, d=d, **MODES[mode]))
    g = gen.rmat(14, 22, weight="f32", wlo=0.5, whi=1.5)
    s = int(gen.random_sources(g, 1, 5)[0])
    assert_solve_parity(g, s, gpu_solve(g, s, **MODES[mode]))


@pytest.mark.parametrize("mode", MODES)
def test_hubs(mode):
    """A hub whose arcs flood the LDS frontier, and a hub with arcs into
    20000 single-vertex partitions (far more distinct heads in one batch
    than the buffer and the wakeup table hold: their overflow paths)."""
    rng = np.random.default_rng(5)
    n = 40001
    u = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(1, n, size=60000)])
    v = np.concatenate([np.arange(1, n), rng.integers(1, n, size=60000)])
    w = rng.integers(1, 50, size=u.size).astype(np.uint32)
    keep = u != v
    g = gen.from_arcs(n, u[keep], v[keep], w[keep])
    for P in (2, 64):
        assert_solve_parity(g, 0, gpu_solve(g, 0, num_partitions=P, delta=1000.0,
                                            **MODES[mode]))
    n = 20001
    rng = np.random.default_rng(6)
    u = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(1, n, size=40000)])
    v = np.concatenate([np.arange(1, n), rng.integers(1, n, size=40000)])
    w = rng.integers(1, 30, size=u.size).astype(np.uint32)
    keep = u != v
    g = gen.from_arcs(n, u[keep], v[keep], w[keep])
    ref = oracle.solve(g.row_ptr, g.col, g.w, 0)
    for kw in (dict(num_partitions=n), dict(num_partitions=4000, delta=-1.0, wg_size=256)):
        assert_solve_parity(g, 0, gpu_solve(g, 0, **kw, **MODES[mode]), ref)


@pytest.mark.parametrize("mode", MODES)
def test_long_path(mode):
    n = 3000
    u = np.arange(n - 1)
    w = np.random.default_rng(3).integers(1, 9, size=n - 1).astype(np.uint32)
    g = gen.from_arcs(n, u, u + 1, w)
    for P in (1, 7):
        assert_solve_parity(g, 0, gpu_solve(g, 0, num_partitions=P, lag=-1, **MODES[mode]))


@pytest.mark.parametrize("mode", MODES)
def test_deterministic_repeats(c1, mode):
    g, d, ref = c1
    s = sssp_mod().Solver(*d, num_partitions=16, **MODES[mode])
    for _ in range(5):
        dist, pred, pe = s(0, sync=True)
        assert_solve_parity(g, 0, (dist.cpu().numpy().view(np.uint32), pred.cpu().numpy(),
                                   pe.cpu().numpy()), ref)


@pytest.mark.parametrize("mode", MODES)
def test_rmat20_full_size_pruned(mode):
    """The headline workload at full size: R-MAT 20 pruned, 256 partitions."""
    g = gen.rmat(20, 20)
    s = int(gen.random_sources(g, 1, 20)[0])
    S = sssp_mod()
    rp, c, w = dev(g)
    keep, (prp, pc, pw, emap) = S.prune(rp, c, w, num_partitions=256)
    solver = S.Solver(prp, pc, pw, num_partitions=256, stats=True, **MODES[mode])
    dist, pred, pe = solver(s, sync=True)
    dist = dist.cpu().numpy().view(np.uint32)
    pe = pe.cpu().numpy()
    emap = emap.cpu().numpy()
    pe_orig = np.where(pe >= 0, emap[np.maximum(pe, 0)], -1)
    assert_solve_parity(g, s, (dist, pred.cpu().numpy(), pe_orig))


@pytest.mark.parametrize("mode", ["buffered"])
def test_grid4096_full_size(mode):
    g = gen.grid(4096, 4096, seed=3)
    dist, pred, pe = gpu_solve(g, 0, **MODES[mode])
    assert oracle.certify(g.row_ptr, g.col, g.w, 0, dist, pe) == (0, -1)
    assert_solve_parity(g, 0, (dist, pred, pe))


@pytest.mark.parametrize("mode", MODES)
def test_batched(mode):
    """A batch of uneven R-MAT graphs (scales 8..14, 3 sources each) in one
    launch, in the mode, against the oracle."""
    rng = np.random.default_rng(11)
    scales = rng.integers(8, 15, size=10)
    graphs = [gen.rmat(int(sc), 6000 + i) for i, sc in enumerate(scales)]
    sg, ss = [], []
    for i, g in enumerate(graphs):
        for s in gen.random_sources(g, 3, 8000 + i):
            sg.append(i)
            ss.append(int(s))
    S = sssp_mod()
    dists, preds, pes = S.solve_batch([dev(g) for g in graphs], sg, ss, **MODES[mode])
    for k, (gi, s) in enumerate(zip(sg, ss)):
        assert_solve_parity(graphs[gi], s, (dists[k].cpu().numpy().view(np.uint32),
                                            preds[k].cpu().numpy(), pes[k].cpu().numpy()))


def test_heap_grid_and_fp32_orders():
    """The heap mode settles a partition in exact distance order, also with
    fp32 costs (which no bucket width orders exactly): a 1024^2 grid, and
    fp32 R-MAT and grid graphs with costs that round, against the fp32
    oracle bit for bit, with one unbounded lag window and with the default."""
    g = gen.grid(1024, 1024, seed=7)
    dist, pred, pe = gpu_solve(g, 0, local_heap=True)
    assert oracle.certify(g.row_ptr, g.col, g.w, 0, dist, pe) == (0, -1)
    assert_solve_parity(g, 0, (dist, pred, pe))
    gf = gen.rmat(15, 31, weight="f32", wlo=0.1, whi=3.0)
    s = int(gen.random_sources(gf, 1, 31)[0])
    ref = oracle.solve(gf.row_ptr, gf.col, gf.w, s)
    for kw in (dict(), dict(lag=-1), dict(num_partitions=7, wg_size=256)):
        assert_solve_parity(gf, s, gpu_solve(gf, s, local_heap=True, **kw), ref)
    gg = gen.grid(300, 200, seed=8, weight="f32", wlo=0.5, whi=1.5)
    assert_solve_parity(gg, 0, gpu_solve(gg, 0, local_heap=True, num_partitions=16))


def test_heap_flag_excludes_buffering():
    S = sssp_mod()
    g = gen.uniform(64, 256, 2)
    with pytest.raises(S.SSSPError) as ei:
        gpu_solve(g, 0, local_heap=True, buffer_cross=True)
    assert ei.value.code == -1


# ------------------------------------------------ idle-time pruning (LOCAL)
def idle_prune_solve(g, s, P, **kw):
    S = sssp_mod()
    rp, c, w = dev(g)
    solver = S.Solver(rp, c, w, num_partitions=P, idle_prune=True, want_keep=True, stats=True,
                      **kw)
    dist, pred, pe = solver(s, sync=True)
    st = solver.stats.read()
    assert st["status"] == 0 and st["num_partitions"] == P
    res = (dist.cpu().numpy().view(np.uint32) if g.w.dtype == np.uint32 else dist.cpu().numpy(),
           pred.cpu().numpy(), pe.cpu().numpy())
    return res, solver.keep[:g.m].cpu().numpy(), st


def check_idle_prune(g, s, P, **kw):
    """Distances and predecessors equal the oracle's on the unpruned graph,
    and every arc deleted during the solve is in the oracle's LOCAL
    deletion set for the same partitions."""
    res, keep, st = idle_prune_solve(g, s, P, **kw)
    assert_solve_parity(g, s, res)
    local_del = oracle.trishla(g.row_ptr, g.col, g.w, local_scope=True, nparts=P) == 0
    deleted = keep == 0
    assert not np.any(deleted & ~local_del), np.nonzero(deleted & ~local_del)[0][:10]
    assert int(deleted.sum()) == st["edges_pruned"]
    return int(deleted.sum()), int(local_del.sum())


@pytest.mark.parametrize("case", ["c1", "rmat14", "rmat13_f32", "rmat14_wg256"])
def test_idle_prune_parity_and_subset(case):
    if case == "c1":
        g, s, P, kw = gen.uniform(4096, 32768, seed=1), 0, 4, {}
    elif case == "rmat13_f32":
        g = gen.rmat(13, 13, weight="f32", wlo=0.1, whi=3.0)
        s, P, kw = int(gen.random_sources(g, 1, 13)[0]), 8, {}
    else:
        g = gen.rmat(14, 14)
        s, P = int(gen.random_sources(g, 1, 14)[0]), 16
        kw = dict(wg_size=256, num_workgroups=64) if case.endswith("wg256") else {}
    check_idle_prune(g, s, P, **kw)


def test_idle_prune_runs_while_the_frontier_is_elsewhere():
    """Partition 0 holds a 4096-vertex path from the source (one vertex per
    round, so the solve takes many batches); partition 1 is a dense random
    cluster reached only through the path's end.  Idle workgroups prune
    partition 1 long before the solve gets there: arcs are deleted, all of
    them in the LOCAL deletion set, and the result is exact."""
    rng = np.random.default_rng(12)
    B = 4096
    pu, pv = np.arange(B - 1), np.arange(1, B)
    m1 = 64 * B
    cu = rng.integers(B, 2 * B, size=m1)
    cv = rng.integers(B, 2 * B, size=m1)
    ok = cu != cv
    u = np.concatenate([pu, [B - 1], cu[ok]])
    v = np.concatenate([pv, [B], cv[ok]])
    w = np.concatenate([np.ones(B, np.uint32), rng.integers(1, 101, size=int(ok.sum()))
                        .astype(np.uint32)])
    g = gen.from_arcs(2 * B, u, v, w)
    pruned, local = check_idle_prune(g, 0, 2, lag=-1)
    assert local > 0 and pruned > 0, (pruned, local)


def test_idle_prune_refused_with_other_modes_and_batches():
    S = sssp_mod()
    g = gen.uniform(64, 256, 2)
    with pytest.raises(S.SSSPError) as ei:
        gpu_solve(g, 0, idle_prune=True, local_heap=True)
    assert ei.value.code == -1
    with pytest.raises(S.SSSPError) as ei:
        S.solve_batch([dev(g)], [0], [0], idle_prune=True)
    assert ei.value.code == -1
