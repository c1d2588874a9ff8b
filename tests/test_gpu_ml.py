"""GPU parity of the multilevel initial bipartitioning (paper Sec. 5.2
"Initial Bipartitioning"; kmp_options.ip_multilevel): whole partitions and a
batch through the C ABI against the CPU oracle with the same options,
bit-exact.  The cases cover several coarsening levels per block, FM on the
finer levels, the pool, the adaptive caps, weighted graphs and rows longer
than one thread's share (hubs)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.helpers import with_hubs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kmp():
    import paper_2105_02022_amd as k
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    k.library()  # raises if libkmp.so is missing: no fallback
    return k


def dev(g):
    import paper_2105_02022_amd as k
    return k.to_device(g, "cuda")


def _cases():
    return [("grid40x50", gen.grid(40, 50), 8),
            ("rgg3000", gen.rgg(3000, 8.0, seed=3), 16),
            ("weighted2000", gen.random_graph(2000, 5.0, 12, max_vw=5, max_ew=7), 7),
            ("rmat12", gen.rmat(12, 8 << 12, seed=9), 64),
            ("rgg20000", gen.rgg(20000, 8.0, seed=5), 64),
            ("rgg8000+hubs", with_hubs(gen.rgg(8000, 6.0, 7), [600, 1500], seed=4), 12)]


@pytest.mark.parametrize("ci", range(6))
@pytest.mark.parametrize("fm,pool,adaptive", [(0, False, False), (2, False, False), (1, True, True)])
def test_partition_multilevel_ip_matches_oracle(kmp, ci, fm, pool, adaptive):
    name, g, k = _cases()[ci]
    say(f"[partition ip_multilevel] {name} k={k} fm={fm} pool={pool} adaptive={adaptive}")
    ref = oracle.partition(g, k, 0.03, 3, fm_passes=fm, pool=pool, adaptive_eps=adaptive, ip_multilevel=True)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, out, st = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 3, fm_passes=fm, ip_pool=pool,
                                       adaptive_eps=adaptive, ip_multilevel=True)
    assert rc == ref.status, name
    assert np.array_equal(out.cpu().numpy(), ref.part), name
    assert st["cut"] == ref.stats["cut"], name


def test_batch_multilevel_ip_matches_oracle(kmp):
    cases = _cases()[:4]
    jobs = []
    for name, g, k in cases:
        xadj, adjncy, vwgt, adjwgt = dev(g)
        jobs.append(dict(xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, k=k, epsilon=0.03, seed=8,
                         out=torch.full((g.n,), -5, dtype=torch.int32, device="cuda")))
    say(f"[batch ip_multilevel] {len(jobs)} jobs")
    rc, res, _ = kmp.kmp_partition_batch(jobs, fm_passes=2, ip_multilevel=True)
    assert rc >= 0
    for (name, g, k), j, r in zip(cases, jobs, res):
        ref = oracle.partition(g, k, 0.03, 8, fm_passes=2, ip_multilevel=True)
        assert r["status"] == ref.status, name
        assert np.array_equal(j["out"].cpu().numpy(), ref.part), name
        assert r["cut"] == ref.stats["cut"], name


def test_multilevel_ip_option_rejected_out_of_range(kmp):
    g = gen.grid(10, 10)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 4, 0.03, 1, ip_multilevel=2)
    assert rc == kmp.KMP_EINVAL
