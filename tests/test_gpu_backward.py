"""GPU parity of the differentiable form: fp32 forward bit-exact against the
fp32 oracle, sssp_backward against the oracle gradient (tree-path
definition) and float64 finite differences, the Euler identity, and scale
invariance."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_12012_amd import gen
from helpers import dev, poison_cached_memory, sssp_mod

pytestmark = pytest.mark.gpu


def setup(scale, seed, ntarget=1024):
    g = gen.rmat(scale, seed, weight="f32", wlo=0.5, whi=1.5)
    s = int(gen.random_sources(g, 1, seed)[0])
    t = gen.random_targets(g, s, ntarget, seed + 1)
    gv = np.zeros(g.n, np.float32)
    gv[t] = 1.0
    return g, s, gv


def gpu_grad(g, s, gv):
    S = sssp_mod()
    rp, c, w = dev(g)
    wt = w.clone().requires_grad_(True)
    d = S.SSSPDist.apply(wt, rp, c, s)
    loss = (d[torch.isfinite(d)] * torch.from_numpy(gv).cuda()[torch.isfinite(d)]).sum()
    loss.backward()
    return d.detach().cpu().numpy(), wt.grad.cpu().numpy(), float(loss)


@pytest.mark.parametrize("scale,seed", [(10, 10), (14, 14)])
def test_forward_and_gradient_match_oracle(scale, seed):
    g, s, gv = setup(scale, seed)
    d, gw, loss = gpu_grad(g, s, gv)
    dref = oracle.sssp(g.row_ptr, g.col, g.w, s)
    assert np.array_equal(d.view(np.uint32), dref.view(np.uint32))
    pe_ref, _ = oracle.pred(g.row_ptr, g.col, g.w, s, dref)
    gref = oracle.grad(g.row_ptr, s, pe_ref, gv)
    np.testing.assert_allclose(gw, gref, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("byte", [0x5A, 0xFF])
def test_gradient_with_stale_workspace_contents(byte):
    """Forward and backward give the oracle's distances and gradient when
    their workspaces and outputs start with a stale byte pattern."""
    g, s, gv = setup(13, 15)
    poison_cached_memory(byte)
    d, gw, loss = gpu_grad(g, s, gv)
    dref = oracle.sssp(g.row_ptr, g.col, g.w, s)
    assert np.array_equal(d.view(np.uint32), dref.view(np.uint32))
    pe_ref, _ = oracle.pred(g.row_ptr, g.col, g.w, s, dref)
    np.testing.assert_allclose(gw, oracle.grad(g.row_ptr, s, pe_ref, gv), rtol=1e-4, atol=1e-4)


def test_gradient_matches_finite_differences_scale10():
    g, s, gv = setup(10, 10)
    d, gw, loss = gpu_grad(g, s, gv)
    edges = np.nonzero(gw)[0]
    rng = np.random.default_rng(0)
    zero = rng.choice(np.nonzero(gw == 0)[0], size=min(200, int((gw == 0).sum())), replace=False)
    sel = np.concatenate([edges, zero])
    fd, valid = oracle.finite_diff(g.row_ptr, g.col, g.w, s, gv, eps=1e-3, edges=sel)
    assert valid.mean() > 0.9
    np.testing.assert_allclose(gw[sel][valid], fd[valid], rtol=1e-4, atol=1e-4)


def test_euler_identity_and_scaling():
    g, s, gv = setup(12, 3)
    d, gw, loss = gpu_grad(g, s, gv)
    lhs = float(np.dot(gw.astype(np.float64), g.w.astype(np.float64)))
    assert abs(lhs - loss) <= 1e-5 * abs(loss)
    g2 = g.with_weights((2 * g.w).astype(np.float32))
    d2, gw2, loss2 = gpu_grad(g2, s, gv)
    assert np.array_equal(d2, 2 * d)
    assert np.array_equal(gw2, gw)


def test_dense_upstream_gradient():
    g = gen.rmat(11, 4, weight="f32", wlo=0.5, whi=1.5)
    s = int(gen.random_sources(g, 1, 4)[0])
    rng = np.random.default_rng(1)
    gv = rng.standard_normal(g.n).astype(np.float32)
    S = sssp_mod()
    rp, c, w = dev(g)
    dist, _, pe = S.solve(rp, c, w, s)
    gw = S.backward(rp, c, w, s, dist, pe, torch.from_numpy(gv).cuda()).cpu().numpy()
    dref = oracle.sssp(g.row_ptr, g.col, g.w, s)
    pe_ref, _ = oracle.pred(g.row_ptr, g.col, g.w, s, dref)
    gv_reached = np.where(np.isfinite(dref), gv, 0).astype(np.float32)
    np.testing.assert_allclose(gw, oracle.grad(g.row_ptr, s, pe_ref, gv_reached),
                               rtol=1e-4, atol=1e-4)


def test_rmat22_full_size_gradient():
    """The differentiable workload at full size: R-MAT scale 22, fp32
    weights, loss = sum of distances to 1024 reachable targets."""
    g, s, gv = setup(22, 22)
    d, gw, loss = gpu_grad(g, s, gv)
    dref = oracle.sssp(g.row_ptr, g.col, g.w, s)
    assert np.array_equal(d.view(np.uint32), dref.view(np.uint32))
    pe_ref, _ = oracle.pred(g.row_ptr, g.col, g.w, s, dref)
    np.testing.assert_allclose(gw, oracle.grad(g.row_ptr, s, pe_ref, gv), rtol=1e-4, atol=1e-4)
