"""sssp_autotune: the chosen options are valid, caller-fixed fields stay
fixed, the JSON cache is written, and solves with the tuned and with the
automatic (cache-consulting) options keep bit-exact parity."""
import json

import pytest

from paper_2103_12012_amd import gen
from helpers import assert_solve_parity, dev, gpu_solve, sssp_mod

pytestmark = pytest.mark.gpu


def test_autotune_then_solve(tmp_path):
    g = gen.rmat(12, 31)
    s = int(gen.random_sources(g, 1, 31)[0])
    S = sssp_mod()
    d = dev(g)
    path = tmp_path / "tune.json"
    best = S.autotune(*d, s, cache_path=str(path))
    assert best["num_partitions"] >= 1 and best["wg_size"] in (256, 512)
    assert best["delta"] == -1.0 or best["delta"] >= 0  # 0 = the automatic width
    text = path.read_text()
    entries = json.loads(text)
    assert any("log2n=12" in e["key"] for e in entries)
    assert_solve_parity(g, s, gpu_solve(g, s, d, **best))
    # automatic options now come from the cache
    assert_solve_parity(g, s, gpu_solve(g, s, d))
    s2 = int(gen.random_sources(g, 2, 77)[1])
    assert_solve_parity(g, s2, gpu_solve(g, s2, d))


def test_autotune_keeps_fixed_fields():
    g = gen.uniform(3000, 24000, 5)
    S = sssp_mod()
    d = dev(g)
    best = S.autotune(*d, 0, num_partitions=7, lag=1, wg_size=512)
    assert best["num_partitions"] == 7 and best["lag"] == 1 and best["wg_size"] == 512
    assert_solve_parity(g, 0, gpu_solve(g, 0, d, **best))


def test_autotune_fp32():
    g = gen.rmat(11, 8, weight="f32")
    s = int(gen.random_sources(g, 1, 8)[0])
    S = sssp_mod()
    d = dev(g)
    best = S.autotune(*d, s)
    assert_solve_parity(g, s, gpu_solve(g, s, d, **best))
