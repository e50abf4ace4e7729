"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare with the oracle on the same seeded inputs."""
import numpy as np

import oracle
from paper_2103_12012_amd import gen


def sssp_mod():
    from paper_2103_12012_amd import sssp

    return sssp


def dev(g):
    return sssp_mod().to_device(g, "cuda")


def host_dist(t, wtype):
    a = t.detach().cpu().numpy()
    return a.view(np.uint32) if wtype == np.uint32 else a


def gpu_solve(g, source, d=None, **kw):
    """(dist, pred, pred_edge) from sssp_solve as numpy arrays."""
    rp, c, w = d if d is not None else dev(g)
    dist, pred, pe = sssp_mod().solve(rp, c, w, int(source), **kw)
    return host_dist(dist, g.w.dtype), pred.cpu().numpy(), pe.cpu().numpy()


def assert_solve_parity(g, source, res, ref=None):
    dist, pred, pe = res
    dr, pr, per = ref if ref is not None else oracle.solve(g.row_ptr, g.col, g.w, int(source))
    if g.w.dtype == np.float32:
        assert np.array_equal(dist.view(np.uint32), dr.view(np.uint32)), \
            f"fp32 dist differs at {np.nonzero(dist.view(np.uint32) != dr.view(np.uint32))[0][:10]}"
    else:
        bad = np.nonzero(dist != dr)[0]
        assert bad.size == 0, f"dist differs at {bad[:10]}: gpu {dist[bad[:5]]} ref {dr[bad[:5]]}"
    bad = np.nonzero(pe != per)[0]
    assert bad.size == 0, f"pred_edge differs at {bad[:10]}: gpu {pe[bad[:5]]} ref {per[bad[:5]]}"
    assert np.array_equal(pred, pr)


def tiny_graph(seed, n=None, m=None, wmax=5, zero=True, loops=True):
    rng = np.random.default_rng(seed)
    n = n or int(rng.integers(1, 65))
    m = m if m is not None else int(rng.integers(0, 4 * n + 1))
    u = rng.integers(0, n, size=m)
    v = rng.integers(0, n, size=m)
    if not loops:
        keep = u != v
        u, v = u[keep], v[keep]
    w = rng.integers(0 if zero else 1, wmax + 1, size=u.shape[0]).astype(np.uint32)
    return gen.from_arcs(n, u, v, w)


def poison_cached_memory(byte, nbytes=1 << 30):
    """Leave `nbytes` of device memory filled with `byte` in torch's caching
    allocator, so the next allocations (workspaces, outputs) start with that
    pattern instead of fresh zeroed pages."""
    import torch

    torch.cuda.synchronize()
    junk = torch.full((nbytes,), byte, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    del junk

