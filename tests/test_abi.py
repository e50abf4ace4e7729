"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments on the host before touching the device."""
import ctypes

import pytest

from paper_2103_12012_amd import sssp

L = None


@pytest.fixture(scope="module")
def lib():
    return sssp.lib()


def fake_csr(n=10, m=20, wtype=sssp.W_U32):
    # pointers are never dereferenced on the host-side paths exercised here
    return sssp.CSR(n, m, 0x1000, 0x2000, 0x3000, wtype, 0)


def ws_query(lib, g, source=0, opts=None):
    nb = ctypes.c_size_t(0)
    o = opts or sssp.make_opts()
    rc = lib.sssp_solve(ctypes.byref(g), source, ctypes.byref(o), None, None, None, None,
                        None, ctypes.byref(nb), None)
    return rc, nb.value


def test_exports_every_declared_symbol(lib):
    names = sssp.declared_symbols()
    assert set(names) >= {"sssp_prune", "sssp_solve", "sssp_solve_batch", "sssp_backward",
                          "sssp_strerror", "sssp_autotune", "sssp_autotune_batch", "sssp_opts_init",
                          "sssp_version", "sssp_solve_noalloc"}
    for s in names:
        assert hasattr(lib, s), s


def test_strerror_and_version(lib):
    for code in sssp.ERRORS:
        assert sssp.strerror(code)
    assert sssp.strerror(12345) == "unknown error"
    assert "gfx950" in sssp.version()


def test_opts_init(lib):
    o = sssp.Opts()
    o.delta, o.flags, o.wg_size = 3.0, 7, 512
    lib.sssp_opts_init(ctypes.byref(o))
    assert o.delta == 0 and o.flags == 0 and o.wg_size == 0 and o.event_start is None


def test_struct_sizes():
    assert ctypes.sizeof(sssp.CSR) == 40
    assert ctypes.sizeof(sssp.Opts) == 56
    assert ctypes.sizeof(sssp.Stats) == 120


def test_solve_host_errors(lib):
    assert ws_query(lib, fake_csr())[0] == 0
    assert ws_query(lib, fake_csr(n=0))[0] == -1
    assert ws_query(lib, fake_csr(m=-1))[0] == -1
    assert ws_query(lib, fake_csr(m=2**31 - 2**24))[0] == 0  # SSSP_M_MAX
    assert ws_query(lib, fake_csr(m=2**31 - 2**24 + 1))[0] == -1
    assert ws_query(lib, fake_csr(n=2**30 - 2**24))[0] == 0  # SSSP_N_MAX
    assert ws_query(lib, fake_csr(n=2**30 - 2**24 + 1))[0] == -1
    assert ws_query(lib, fake_csr(wtype=5))[0] == -1
    g = fake_csr()
    g.row_ptr = None
    assert ws_query(lib, g)[0] == -1
    g = fake_csr()
    g.reserved = 1
    assert ws_query(lib, g)[0] == -1
    assert ws_query(lib, fake_csr(), source=-1)[0] == -2
    assert ws_query(lib, fake_csr(), source=10)[0] == -2
    assert ws_query(lib, fake_csr(), opts=sssp.make_opts(wg_size=100))[0] == -1
    assert ws_query(lib, fake_csr(), opts=sssp.make_opts(delta=float("nan")))[0] == -1
    assert ws_query(lib, fake_csr(), opts=sssp.make_opts(num_partitions=-2))[0] == -1
    assert ws_query(lib, fake_csr(), opts=sssp.make_opts(max_rounds=-1))[0] == -1
    assert lib.sssp_solve(None, 0, None, None, None, None, None, None, None, None) == -1
    g = fake_csr()
    assert lib.sssp_solve(ctypes.byref(g), 0, None, None, None, None, None, None, None,
                          None) == -1  # ws_bytes NULL


def test_workspace_size_grows_and_is_checked(lib):
    _, small = ws_query(lib, fake_csr(n=1000, m=100))
    _, big = ws_query(lib, fake_csr(n=100000, m=100))
    assert 0 < small < big
    g = fake_csr(n=1000, m=100)
    o = sssp.make_opts()
    dist = ctypes.c_void_p(0x4000)
    nb = ctypes.c_size_t(small - 256)
    buf = ctypes.c_void_p(0x10000)
    assert lib.sssp_solve(ctypes.byref(g), 0, ctypes.byref(o), dist, None, None, None, buf,
                          ctypes.byref(nb), None) == -9
    nb = ctypes.c_size_t(small)
    misaligned = ctypes.c_void_p(0x10010)
    assert lib.sssp_solve(ctypes.byref(g), 0, ctypes.byref(o), dist, None, None, None,
                          misaligned, ctypes.byref(nb), None) == -9
    # missing dist output
    assert lib.sssp_solve(ctypes.byref(g), 0, ctypes.byref(o), None, None, None, None, buf,
                          ctypes.byref(nb), None) == -1


def test_prune_host_errors(lib):
    g = fake_csr()
    o = sssp.make_opts()
    nb = ctypes.c_size_t(0)
    assert lib.sssp_prune(ctypes.byref(g), ctypes.byref(o), None, None, None, None, None, None,
                          None, ctypes.byref(nb), None) == 0 and nb.value > 0
    # compaction outputs must be all set or all NULL
    p = ctypes.c_void_p(0x5000)
    assert lib.sssp_prune(ctypes.byref(g), ctypes.byref(o), None, p, None, None, None, None,
                          None, ctypes.byref(nb), None) == -1
    nb2 = ctypes.c_size_t(0)
    assert lib.sssp_prune(ctypes.byref(g), ctypes.byref(o), None, p, p, p, p, None, None,
                          ctypes.byref(nb2), None) == 0 and nb2.value > nb.value


def test_backward_host_errors(lib):
    o = sssp.make_opts()
    nb = ctypes.c_size_t(0)
    g = fake_csr(wtype=sssp.W_U32)
    assert lib.sssp_backward(ctypes.byref(g), 0, None, None, None, None, ctypes.byref(o), None,
                             None, ctypes.byref(nb), None) == -1
    g = fake_csr(wtype=sssp.W_F32)
    assert lib.sssp_backward(ctypes.byref(g), 0, None, None, None, None, ctypes.byref(o), None,
                             None, ctypes.byref(nb), None) == 0 and nb.value > 0
    assert lib.sssp_backward(ctypes.byref(g), 11, None, None, None, None, ctypes.byref(o),
                             None, None, ctypes.byref(nb), None) == -2


def test_batch_host_errors(lib):
    gs = (sssp.CSR * 2)(fake_csr(n=10), fake_csr(n=20))
    sg = (ctypes.c_int32 * 3)(0, 1, 1)
    ss = (ctypes.c_int32 * 3)(0, 5, 19)
    off = (ctypes.c_int64 * 3)(0, 10, 30)
    o = sssp.make_opts()
    nb = ctypes.c_size_t(0)
    args = lambda n_s=3, sg=sg, ss=ss: lib.sssp_solve_batch(
        2, gs, n_s, sg, ss, off, ctypes.byref(o), None, None, None, None, None,
        ctypes.byref(nb), None)
    assert args() == 0 and nb.value > 0
    assert args(n_s=0) == -1
    assert args(sg=(ctypes.c_int32 * 3)(0, 2, 1)) == -1
    assert args(ss=(ctypes.c_int32 * 3)(0, 5, 20)) == -2
    gs[1].wtype = sssp.W_F32
    assert args() == -1


def test_autotune_batch_host_errors(lib):
    """Argument errors of sssp_autotune_batch are found on the host."""
    g = sssp.CSR()
    g.n, g.m, g.wtype = 4, 0, 0
    nb = ctypes.c_size_t(0)
    sg = (ctypes.c_int32 * 1)(0)
    ss = (ctypes.c_int32 * 1)(0)
    off = (ctypes.c_int64 * 1)(0)
    o = sssp.make_opts(validate=False)
    # no best options
    assert lib.sssp_autotune_batch(1, ctypes.byref(g), 1, sg, ss, off, None, None, None, None,
                                   ctypes.byref(nb), None) == -1
    # no graphs
    assert lib.sssp_autotune_batch(0, ctypes.byref(g), 1, sg, ss, off, None, ctypes.byref(o),
                                   None, None, ctypes.byref(nb), None) == -1


def test_noalloc_rejects_graphs_beyond_the_fixed_workspace(lib):
    """sssp_solve_noalloc refuses, on the host, a graph whose solve needs more
    than SSSP_NOALLOC_SCRATCH_BYTES (the pointers are never dereferenced)."""
    limit = 64 << 20
    g = fake_csr(n=9_000_000, m=100)
    _, need = ws_query(lib, g)
    assert need > limit
    assert lib.sssp_solve_noalloc(ctypes.byref(g), 0, None, ctypes.c_void_p(0x4000), None,
                                  None, None, None) == -13
    assert lib.sssp_solve_noalloc(ctypes.byref(g), -1, None, ctypes.c_void_p(0x4000), None,
                                  None, None, None) == -2
    _, need = ws_query(lib, fake_csr(n=7_000_000, m=100))
    assert need <= limit
