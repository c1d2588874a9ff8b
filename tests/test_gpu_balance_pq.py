"""GPU parity of the queue balancer (kmp_options.pq_balance, paper Sec. 5.3
Balancing): the balancing step alone through kmp_balance_ex against the
oracle's queue balancer on the cases its pins use, and whole partitions and
batches whose levels need balancing (heavy nodes), bit-exact."""
import sys

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.test_oracle_pins_pq import _case

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


def dev(g):
    import paper_2105_02022_amd as k
    return k.to_device(g, "cuda")


@pytest.mark.parametrize("seed", list(range(12)) + [33, 54, 66, 81, 144])
def test_balance_step_pq(kmp, seed):
    g, part, wt, cap = _case(seed, max_vw=1 + seed % 4)
    say(f"[pq balance step] seed={seed} n={g.n} nb={len(wt)}")
    exp_part, exp_wt, exp_p = oracle.balance_pq(g, seed % 3, 900 + seed, part, wt, cap)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    d_part = torch.from_numpy(part.copy()).cuda()
    d_wt = torch.from_numpy(wt.copy()).cuda()
    d_cap = torch.from_numpy(cap.copy()).cuda()
    r = kmp.kmp_balance_ex(xadj, adjncy, vwgt, adjwgt, seed % 3, 900 + seed, d_part, d_wt, d_cap, pq=True)
    assert r == exp_p
    assert np.array_equal(d_part.cpu().numpy(), exp_part)
    assert np.array_equal(d_wt.cpu().numpy(), exp_wt)


def test_balance_step_pq_larger(kmp):
    for seed in range(3):
        g, part, wt, cap = _case(100 + seed, n=3000, nb=9, max_vw=5, iso=0.05)
        say(f"[pq balance step] n=3000 seed={seed}")
        exp_part, exp_wt, exp_p = oracle.balance_pq(g, 1, seed, part, wt, cap)
        xadj, adjncy, vwgt, adjwgt = dev(g)
        d_part = torch.from_numpy(part.copy()).cuda()
        d_wt = torch.from_numpy(wt.copy()).cuda()
        d_cap = torch.from_numpy(cap.copy()).cuda()
        r = kmp.kmp_balance_ex(xadj, adjncy, vwgt, adjwgt, 1, seed, d_part, d_wt, d_cap, pq=True)
        assert r == exp_p
        assert np.array_equal(d_part.cpu().numpy(), exp_part)


def _heavy(n, seed, frac=0.15, w=40):
    g = gen.random_graph(n, 5.0, seed)
    g.vwgt = np.where(np.random.default_rng(seed + 7).random(n) < frac, w, 1).astype(np.int32)
    return g


# heavy-node inputs on which the balancer runs (several passes, and a final imbalance on the last two)
@pytest.mark.parametrize("name,k", [("heavy9000", 33), ("heavy8000", 50), ("heavy12000", 64), ("heavy3000", 16),
                                    ("rgg20000", 64)])
def test_partition_pq_balance(kmp, name, k):
    g = {"heavy9000": lambda: _heavy(9000, 5, 0.05, 200), "heavy8000": lambda: _heavy(8000, 5, 0.1, 150),
         "heavy12000": lambda: _heavy(12000, 8, 0.05, 250), "heavy3000": lambda: _heavy(3000, 7, 0.02, 800),
         "rgg20000": lambda: gen.rgg(20000, 8.0, 2)}[name]()
    say(f"[pq balance partition] {name} k={k}")
    ref = oracle.partition(g, k, 0.03, 1, pq_balance=True)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, part, st = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 1, pq_balance=True)
    assert rc == ref.status
    assert np.array_equal(part.cpu().numpy(), ref.part)
    assert st["cut"] == ref.stats["cut"] and st["balance_rounds"] == ref.stats["balance_rounds"]


def test_batch_pq_balance(kmp):
    specs = [(_heavy(8000, 5, 0.1, 150), 50, 1), (gen.grid(40, 50), 4, 2), (_heavy(12000, 8, 0.05, 250), 64, 1)]
    jobs = []
    for g, k, seed in specs:
        xadj, adjncy, vwgt, adjwgt = dev(g)
        jobs.append(dict(xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, k=k, epsilon=0.03, seed=seed,
                         out=torch.empty(g.n, dtype=torch.int32, device="cuda")))
    say("[pq balance batch] 3 jobs")
    rc, res, _ = kmp.kmp_partition_batch(jobs, pq_balance=True)
    assert rc == 0
    for (g, k, seed), j, r in zip(specs, jobs, res):
        ref = oracle.partition(g, k, 0.03, seed, pq_balance=True)
        assert r["status"] == ref.status and r["cut"] == ref.stats["cut"]
        assert np.array_equal(j["out"].cpu().numpy(), ref.part)



