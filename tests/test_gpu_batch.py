"""GPU parity of sssp_solve_batch: every (graph, source) result equals the
single-source oracle bit-exactly, independent of batch order, and a
captured HIP graph of the batched call replays correctly."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_12012_amd import gen
from helpers import assert_solve_parity, dev, poison_cached_memory, sssp_mod

pytestmark = pytest.mark.gpu


def make_batch(ngraphs, smin, smax, seed, per_graph=2):
    rng = np.random.default_rng(seed)
    scales = rng.integers(smin, smax + 1, size=ngraphs)
    graphs = [gen.rmat(int(sc), 4000 + seed * 100 + i) for i, sc in enumerate(scales)]
    sg, ss = [], []
    for i, g in enumerate(graphs):
        for s in gen.random_sources(g, per_graph, 7000 + i):
            sg.append(i)
            ss.append(int(s))
    return graphs, sg, ss


def check(graphs, sg, ss, res):
    dists, preds, pes = res
    for k, (gi, s) in enumerate(zip(sg, ss)):
        g = graphs[gi]
        assert_solve_parity(g, s, (dists[k].cpu().numpy().view(np.uint32),
                                   preds[k].cpu().numpy(), pes[k].cpu().numpy()))


def test_batch_equals_single_solves():
    graphs, sg, ss = make_batch(8, 8, 12, seed=1)
    S = sssp_mod()
    dg = [dev(g) for g in graphs]
    check(graphs, sg, ss, S.solve_batch(dg, sg, ss))


def test_batch_order_invariant():
    graphs, sg, ss = make_batch(5, 9, 11, seed=2, per_graph=3)
    S = sssp_mod()
    dg = [dev(g) for g in graphs]
    perm = np.random.default_rng(0).permutation(len(sg))
    sg2 = [sg[i] for i in perm]
    ss2 = [ss[i] for i in perm]
    check(graphs, sg2, ss2, S.solve_batch(dg, sg2, ss2, num_partitions=3))


def test_batch_mixed_sizes_and_tiny():
    graphs = [gen.from_arcs(1, [], [], np.zeros(0, np.uint32)), gen.uniform(300, 1200, 5),
              gen.rmat(13, 9)]
    sg = [0, 1, 2, 1, 2]
    ss = [0, 5, int(gen.random_sources(graphs[2], 1, 1)[0]), 299, 0]
    S = sssp_mod()
    check(graphs, sg, ss, S.solve_batch([dev(g) for g in graphs], sg, ss))


@pytest.mark.parametrize("byte", [0x5A, 0xFF])
def test_batch_with_stale_workspace_contents(byte):
    """The batched launch's workspace and outputs start with whatever the
    allocator's cached memory held (a byte pattern here); results still
    equal the oracle's."""
    graphs, sg, ss = make_batch(6, 9, 13, seed=5)
    S = sssp_mod()
    dg = [dev(g) for g in graphs]
    poison_cached_memory(byte)
    check(graphs, sg, ss, S.solve_batch(dg, sg, ss))


def test_batch_hip_graph_replays():
    graphs, sg, ss = make_batch(6, 8, 11, seed=3)
    S = sssp_mod()
    dg = [dev(g) for g in graphs]
    b = S.BatchSolver(dg, sg, ss)
    b()  # warm-up outside capture
    torch.cuda.synchronize()
    eager = b.dist.clone()
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            b()
    torch.cuda.synchronize()
    for _ in range(4):
        b.dist.fill_(0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.dist, eager)
        check(graphs, sg, ss, (b.split(b.dist), b.split(b.pred), b.split(b.pred_edge)))


def test_batch_autotune_then_parity(tmp_path):
    """sssp_autotune_batch: valid options, a cache entry under the batch
    signature, and the tuned (automatic) launch keeps bit-exact parity."""
    graphs, sg, ss = make_batch(4, 8, 10, seed=5)
    S = sssp_mod()
    dg = [dev(g) for g in graphs]
    b = S.BatchSolver(dg, sg, ss)
    path = tmp_path / "batch.json"
    best = b.autotune(cache_path=str(path))
    assert best["wg_size"] in (256, 512) and best["num_partitions"] >= 0
    assert "|batch|" in path.read_text()
    b()
    torch.cuda.synchronize()
    check(graphs, sg, ss, (b.split(b.dist), b.split(b.pred), b.split(b.pred_edge)))


@pytest.mark.parametrize("buffer_cross", [False, True])
def test_c4_full_size_batched_launch(buffer_cross):
    """The batched workload at full size, as the benchmark runs it: 64 R-MAT
    graphs of scales 12..18 (seed 4, graph i seed 4000+i), 4 random sources
    each, tuned as a whole and launched once through a captured HIP graph;
    every one of the 256 results equals the single-source oracle (also with
    buffered cross-partition updates)."""
    rng = np.random.default_rng(4)
    scales = rng.integers(12, 19, size=64)
    graphs = [gen.rmat(int(sc), 4000 + i) for i, sc in enumerate(scales)]
    sg, ss = [], []
    for i, g in enumerate(graphs):
        for s in gen.random_sources(g, 4, 5000 + i):
            sg.append(i)
            ss.append(int(s))
    S = sssp_mod()
    dg = [dev(g) for g in graphs]
    b = S.BatchSolver(dg, sg, ss, buffer_cross=buffer_cross)
    b.autotune()
    b()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            b()
    torch.cuda.synchronize()
    b.dist.fill_(0)
    graph.replay()
    torch.cuda.synchronize()
    check(graphs, sg, ss, (b.split(b.dist), b.split(b.pred), b.split(b.pred_edge)))
