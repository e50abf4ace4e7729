"""sssp_solve_noalloc (the solve with the library's fixed per-GPU workspace)
against sssp_solve on the same inputs, through the C ABI: several calls in a
row on one GPU, each on a smaller graph than the one before (the fixed
array keeps the previous call's contents), all bit-exact against
sssp_solve's distances, predecessors and predecessor arcs."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2103_12012_amd import gen
from helpers import assert_solve_parity, dev, sssp_mod

pytestmark = pytest.mark.gpu


def noalloc(g, d, source, sync=False, **kw):
    S = sssp_mod()
    rp, c, w = d
    csr = S._csr(rp, c, w)
    o = S.make_opts(sync=sync, **kw)
    # the outputs are the caller's; only the workspace comes from the library
    dist = torch.full((g.n,), -7, dtype=w.dtype, device="cuda")
    pred = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    pe = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    stats = S.StatsBuffer.new("cuda")
    rc = S.lib().sssp_solve_noalloc(ctypes.byref(csr), int(source), ctypes.byref(o),
                                    S._ptr(dist), S._ptr(pred), S._ptr(pe), S._ptr(stats.t),
                                    S._stream())
    assert rc == 0, S.strerror(rc)
    torch.cuda.synchronize()
    assert stats.read()["status"] == 0
    return dist, pred, pe


def host(t):
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.int32 else a


def same_as_solve(g, d, source, **kw):
    S = sssp_mod()
    ref = S.solve(*d, int(source), **kw)
    out = noalloc(g, d, source, **kw)
    for a, b in zip(out, ref):
        assert np.array_equal(host(a), host(b))
    return tuple(host(t) if i == 0 else t.cpu().numpy() for i, t in enumerate(out))


def test_noalloc_matches_solve_on_shrinking_inputs():
    # 4.2M-vertex grid (34 MB of the 64 MiB array), then smaller graphs
    big = gen.grid(2048, 2048, seed=5)
    same_as_solve(big, dev(big), 0)
    r14 = gen.rmat(14, 14)
    s14 = int(gen.random_sources(r14, 1, 14)[0])
    res = same_as_solve(r14, dev(r14), s14, num_partitions=16)
    assert_solve_parity(r14, s14, res)
    c1 = gen.uniform(4096, 32768, seed=1)
    res = same_as_solve(c1, dev(c1), 0, num_partitions=4)
    assert_solve_parity(c1, 0, res)
    f = gen.rmat(11, 3, weight="f32", wlo=0.5, whi=1.5)
    sf = int(gen.random_sources(f, 1, 3)[0])
    res = same_as_solve(f, dev(f), sf)
    assert_solve_parity(f, sf, res)
    one = gen.from_arcs(1, [], [], np.zeros(0, np.uint32))
    res = same_as_solve(one, dev(one), 0)
    assert res[0].tolist() == [0] and res[2].tolist() == [-1]


def test_noalloc_sync_status_and_too_large():
    S = sssp_mod()
    # SSSP_F_SYNC returns the device status (an overflow here)
    g = gen.from_arcs(3, [0, 1], [1, 2], np.array([0xF0000000, 0x20000000], np.uint32))
    rp, c, w = dev(g)
    csr = S._csr(rp, c, w)
    o = S.make_opts(sync=True)
    out = [torch.empty(3, dtype=t, device="cuda") for t in (torch.int32,) * 3]
    rc = S.lib().sssp_solve_noalloc(ctypes.byref(csr), 0, ctypes.byref(o),
                                    *[S._ptr(t) for t in out], None, S._stream())
    assert rc == -7
    # a graph whose workspace exceeds the array is refused before any launch
    fake = S.CSR(9_000_000, 100, 0x1000, 0x2000, 0x3000, S.W_U32, 0)
    rc = S.lib().sssp_solve_noalloc(ctypes.byref(fake), 0, None, ctypes.c_void_p(0x4000),
                                    None, None, None, S._stream())
    assert rc == -13
    # and a good call afterwards still matches sssp_solve
    c1 = gen.uniform(1000, 5000, seed=2)
    same_as_solve(c1, dev(c1), 3)
