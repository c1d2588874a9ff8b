"""GPU: kmp_partition_noalloc, the entry point that allocates nothing (its
device buffers are carved from the library's fixed scratch region), against
kmp_partition_ex on the same inputs: identical partition, cut and status,
on two calls in a row with the second input smaller, up to the stated
limits, with the initial-bipartitioning options, and the region's use
reported within its size."""
import sys

import numpy as np
import pytest

from paper_2105_02022_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kmp():
    import paper_2105_02022_amd as k
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    k.library()
    return k


def _weighted(n, seed):
    return gen.random_graph(n, 6.0, seed, max_vw=5, max_ew=7, isolated_frac=0.05)


GRAPHS = {
    "grid256": lambda: gen.grid(256, 256),                 # n at the limit
    "rgg65536_d15": lambda: gen.rgg(65536, 15.0, 5),       # m close to the limit
    "rmat16": lambda: gen.rmat(16, 1 << 19, seed=3),       # skewed degrees, isolated nodes
    "weighted50000": lambda: _weighted(50000, 9),
    "grid40x50": lambda: gen.grid(40, 50),
    "rgg3000": lambda: gen.rgg(3000, 8.0, 2),
}


def _both(kmp, g, k, seed, **opt):
    xadj, adjncy, vwgt, adjwgt = kmp.to_device(g, "cuda")
    out_na = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    rc_na, _, st_na = kmp.kmp_partition_noalloc(xadj, adjncy, vwgt, adjwgt, k, 0.03, seed, out=out_na, **opt)
    rc, part, st = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, seed, **opt)
    assert rc_na == rc, (rc_na, rc)
    assert torch.equal(out_na, part)
    assert st_na["cut"] == st["cut"] and st_na["level_n"] == st["level_n"]
    assert 0 < st_na["workspace_bytes"] <= kmp.NOALLOC_SCRATCH_BYTES
    return st_na["workspace_bytes"], st["workspace_bytes"]


@pytest.mark.parametrize("first,second,k", [
    ("grid256", "grid40x50", 64), ("rgg65536_d15", "rgg3000", 16), ("rmat16", "grid40x50", 4096),
    ("weighted50000", "rgg3000", 7),
])
def test_noalloc_equals_partition_two_calls(kmp, first, second, k):
    for name, seed in ((first, 1), (second, 2)):
        g = GRAPHS[name]()
        assert g.n <= kmp.NOALLOC_MAX_N and g.m <= kmp.NOALLOC_MAX_M
        say(f"[noalloc] {name} n={g.n} m={g.m} k={k} seed={seed}")
        used, pooled = _both(kmp, g, k, seed)
        say(f"  scratch used {used / 2**20:.1f} MiB (pool path {pooled / 2**20:.1f} MiB)")


def test_noalloc_with_ip_options_and_validation(kmp):
    for name, k in (("rgg65536_d15", 64), ("rmat16", 4096), ("grid40x50", 8)):
        g = GRAPHS[name]()
        say(f"[noalloc options] {name} k={k} fm_passes=2 ip_pool=1 validate=1")
        used, _ = _both(kmp, g, k, 3, fm_passes=2, ip_pool=True, validate=True)
        say(f"  scratch used {used / 2**20:.1f} MiB")


def test_noalloc_rejects_beyond_limits(kmp):
    g = gen.grid(257, 256)  # n = 65792 > limit
    xadj, adjncy, vwgt, adjwgt = kmp.to_device(g, "cuda")
    out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    rc, _, _ = kmp.kmp_partition_noalloc(xadj, adjncy, vwgt, adjwgt, 8, 0.03, 1, out=out)
    assert rc == kmp.KMP_ETOOLARGE
    assert (out == -7).all()
    # the next call within the limits is unaffected
    g = GRAPHS["grid40x50"]()
    _both(kmp, g, 8, 1)
