"""GPU: the CF cache (CFCache plugin, AWP framework section) in memory and on
disk.  A table loaded from disk must be the built table byte for byte, and
grid the same data to the same grid (up to the rounding order of the atomic
flushes of tiles that several chunks share); the cache hits, evicts least
recently used tables past its budget, reloads them from disk, precomputes
and grows, and rebuilds a table whose file is damaged."""

import os

import numpy as np
import pytest

import synth
from oracle.cfbuild import TERM_PS, TERM_W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import cfcache as C  # noqa: E402
from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402


def small(seed=140, n_w=3, h_max=4):
    return synth.tiny_workload(n_ant=8, n_time=20, nchan=3, nx=96, ny=80, oversample=8,
                               terms=TERM_PS | TERM_W, n_w=n_w, h_min=2, h_max=h_max,
                               cfg_id=seed)


def specs(wl, p):
    return W.grid_spec(wl.grid), W.cf_spec(wl.cf, p)


# two gridding runs differ only in the order of atomic adds
SAME = {"f64": 1e-13, "f32": 1e-6, "f16cf": 1e-6, "bf16cf": 1e-6}


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def grid_with(cf, wl, p):
    v = W.device_vis(wl, p)
    g = W.empty_grid(wl, p)
    lr.lr_grid(cf, v, p, g)
    torch.cuda.synchronize()
    return g.cpu().numpy()


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf", "bf16cf"])
def test_loaded_table_is_the_built_table(tmp_path, form):
    p = lr.PRECISIONS[form]
    wl = small()
    g, s = specs(wl, p)
    c1 = C.CFCache(str(tmp_path))
    built = c1.get(g, s)
    assert c1.stats["builds"] == 1 and c1.stats["saves"] == 1
    assert os.path.exists(c1.path(C.cf_key(g, s)))
    assert c1.get(g, s) is built and c1.stats["hits"] == 1
    c2 = C.CFCache(str(tmp_path))
    loaded = c2.get(g, s)
    assert c2.stats["loads"] == 1 and c2.stats["builds"] == 0
    torch.cuda.synchronize()
    assert torch.equal(built.blob, loaded.blob)
    assert rel(grid_with(loaded, wl, p), grid_with(built, wl, p)) <= SAME[form]


def test_budget_eviction_reload_precompute_and_growth(tmp_path):
    p = lr.LR_F32
    a, b, c = small(141), small(142, n_w=4), small(143, n_w=5)
    ga, sa = specs(a, p)
    gb, sb = specs(b, p)
    gc, sc = specs(c, p)
    cache = C.CFCache(str(tmp_path))
    cache.precompute([(ga, sa), (gb, sb)])
    assert cache.stats["builds"] == 2 and len(cache.mem) == 2
    nb = cache.get(gb, sb).nbytes
    # a budget that holds one table: the least recently used one leaves
    small_cache = C.CFCache(str(tmp_path), budget=nb + 1)
    small_cache.get(ga, sa)
    small_cache.get(gb, sb)
    assert small_cache.stats["loads"] == 2 and small_cache.stats["evictions"] == 1
    assert C.cf_key(ga, sa) not in small_cache and C.cf_key(gb, sb) in small_cache
    again = small_cache.get(ga, sa)                 # back from disk, not rebuilt
    assert small_cache.stats["loads"] == 3 and small_cache.stats["builds"] == 0
    torch.cuda.synchronize()
    assert torch.equal(again.blob, cache.get(ga, sa).blob)
    # growth on demand: a new table is built and persisted
    cache.get(gc, sc)
    assert cache.stats["builds"] == 3 and os.path.exists(cache.path(C.cf_key(gc, sc)))


def test_damaged_file_is_rebuilt(tmp_path):
    p = lr.LR_F32
    wl = small(144)
    g, s = specs(wl, p)
    ref = C.CFCache(str(tmp_path)).get(g, s)
    path = C.CFCache(str(tmp_path)).path(C.cf_key(g, s))
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0xFF
    open(path, "wb").write(raw)
    cache = C.CFCache(str(tmp_path))
    cf = cache.get(g, s)
    assert cache.stats["bad_files"] == 1 and cache.stats["builds"] == 1
    torch.cuda.synchronize()
    assert torch.equal(cf.blob, ref.blob)
    fresh = C.CFCache(str(tmp_path))                 # the rewritten file loads again
    fresh.get(g, s)
    assert fresh.stats["loads"] == 1 and fresh.stats["bad_files"] == 0
