"""GPU: error paths forced from the host.  KMP_WORKSPACE_LIMIT caps the device
workspace one call may take, so a call that needs more returns KMP_ENOMEM
(and leaves nothing behind: the next call without the cap is correct)."""
import os
import sys

import numpy as np
import pytest

import oracle
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


@pytest.fixture
def limit():
    def set_(v):
        if v is None:
            os.environ.pop("KMP_WORKSPACE_LIMIT", None)
        else:
            os.environ["KMP_WORKSPACE_LIMIT"] = str(v)
    yield set_
    os.environ.pop("KMP_WORKSPACE_LIMIT", None)


def test_workspace_limit_gives_enomem(kmp, limit):
    g = gen.rgg(6000, 8.0, 3)
    xadj, adjncy, vwgt, adjwgt = kmp.to_device(g, "cuda")
    for cap in (1, 4096, 1 << 16):
        say(f"[enomem] partition rgg6000 k=8 with a workspace cap of {cap} bytes")
        limit(cap)
        rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 8, 0.03, 1)
        assert rc == kmp.KMP_ENOMEM, (cap, rc)
    limit(None)
    rc, part, st = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 8, 0.03, 1)
    ref = oracle.partition(g, 8, 0.03, 1)
    assert rc == ref.status
    assert np.array_equal(part.cpu().numpy(), ref.part)


def test_workspace_limit_batch_and_steps(kmp, limit):
    gs = [gen.grid(40, 50), gen.rgg(3000, 8.0, 4)]
    jobs = []
    for i, g in enumerate(gs):
        xadj, adjncy, vwgt, adjwgt = kmp.to_device(g, "cuda")
        jobs.append(dict(xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, k=4, epsilon=0.03, seed=i,
                         out=torch.empty(g.n, dtype=torch.int32, device="cuda")))
    say("[enomem] batch of two jobs and an LP clustering call with a 4 KiB workspace cap")
    limit(4096)
    rc, _, _ = kmp.kmp_partition_batch(jobs)
    assert rc == kmp.KMP_ENOMEM
    xadj, adjncy, vwgt, adjwgt = kmp.to_device(gs[1], "cuda")
    rounds = kmp.kmp_lp_cluster(xadj, adjncy, vwgt, adjwgt, 0, 40, 1)[0]
    assert rounds == kmp.KMP_ENOMEM
    limit(None)
    rc, res, _ = kmp.kmp_partition_batch(jobs)
    assert rc == kmp.KMP_OK
    for i, (g, j) in enumerate(zip(gs, jobs)):
        ref = oracle.partition(g, 4, 0.03, i)
        assert np.array_equal(j["out"].cpu().numpy(), ref.part)


def test_queue_balancer_flag_range(kmp):
    """The queue balancer flag takes 0 or 1; other values are rejected before any work."""
    g = gen.grid(10, 10)
    xadj, adjncy, vwgt, adjwgt = kmp.to_device(g, "cuda")
    rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 4, 0.03, 1, pq_balance=2)
    assert rc == kmp.KMP_EINVAL
    part = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    wt = torch.tensor([100, 0], dtype=torch.int64, device="cuda")
    cap = torch.tensor([50, 60], dtype=torch.int64, device="cuda")
    assert kmp.kmp_balance_ex(xadj, adjncy, vwgt, adjwgt, 0, 1, part, wt, cap, pq=2) == kmp.KMP_EINVAL
