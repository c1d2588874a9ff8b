"""GPU parity of the initial-bipartitioning options of paper Sec. 5.2: the
2-way FM refinement that can follow every growth, and the pool of BFS and
random growths beside GGG.  Bipartition rounds and whole partitions through
the C ABI against the CPU oracle with the same options, bit-exact."""
import sys

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.helpers import csr_from_dense, node_w, two_cliques

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


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _heavy_nodes(n, seed):
    g = gen.random_graph(n, 4.0, seed)
    g.vwgt = np.where(np.random.default_rng(seed + 1).random(n) < 0.12, 50, 1).astype(np.int32)
    return g


def _one_huge_edge(n, seed):
    """A weighted random graph in which one edge weighs more than 2^30 (half the edge-weight sum still
    fits in int32): FM gain updates of its endpoints pass 2^31 unless they are computed in 64 bits."""
    g = gen.random_graph(n, 5.0, seed, max_ew=3)
    w = np.asarray(g.adjwgt, np.int64).copy()
    xadj, adj = np.asarray(g.xadj), np.asarray(g.adjncy)
    u = int(np.argmax(np.diff(xadj)))
    v = int(adj[xadj[u]])
    w[xadj[u]] = (1 << 30) + 7
    rev = xadj[v] + int(np.nonzero(adj[xadj[v]:xadj[v + 1]] == u)[0][0])
    w[rev] = (1 << 30) + 7
    assert w.sum() // 2 < 2**31 - 1
    g.adjwgt = w.astype(np.int32)
    return g


def _rounds(kmp, g, k, level, seed, passes, name, pool=False):
    lk = oracle.lk(int(node_w(g).sum()), k, 0.03)
    part = np.zeros(g.n, np.int32)
    first, fcount = [0], [k]
    d_part = t32(part)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    while max(fcount) >= 2:
        say(f"[ip bipartition] {name} k={k} passes={passes} pool={pool} blocks={len(first)}")
        part, ef, efc = oracle.bipartition_round(g, level, part, first, fcount, lk, seed, fm_passes=passes,
                                                 pool=pool)
        rc, first, fcount = kmp.kmp_bipartition_round(xadj, adjncy, vwgt, adjwgt, level, d_part, first, fcount, lk,
                                                      seed, fm_passes=passes, ip_pool=int(pool))
        assert rc == 0
        assert first == list(ef) and fcount == list(efc)
        assert np.array_equal(d_part.cpu().numpy(), part)


@pytest.mark.parametrize("k,passes", [(2, 1), (2, 3), (16, 1), (16, 3), (5, 16)])
def test_bipartition_round_fm(kmp, k, passes):
    # k = 2: one block of 4000 nodes (global scratch, 64-bit keys); k = 16: down to LDS-sized blocks
    _rounds(kmp, gen.rgg(4000, 8.0, 21), k, 0, 3, passes, "rgg4000")


@pytest.mark.parametrize("name", ["weighted", "heavy", "heavy-lds-and-global", "dense-hybrid", "big-edge-weights",
                                  "edge-above-2^30", "cliques", "tiny", "isolated", "path"])
def test_bipartition_fm_weighted_and_degenerate(kmp, name):
    g, k = {
        "weighted": lambda: (gen.random_graph(900, 5.0, 31, max_vw=20, max_ew=5), 7),
        "heavy": lambda: (_heavy_nodes(300, 33), 4),
        "heavy-lds-and-global": lambda: (_heavy_nodes(3000, 35), 6),
        # many internal entries per block: keys in LDS, entries in global memory (then LDS as blocks shrink)
        "dense-hybrid": lambda: (gen.random_graph(1200, 48.0, 38, max_ew=3), 5),
        # weighted degrees beyond 2^19: the 64-bit keys inside LDS-sized blocks
        "big-edge-weights": lambda: (gen.random_graph(400, 5.0, 36, max_ew=300000), 4),
        "edge-above-2^30": lambda: (_one_huge_edge(400, 37), 4),
        "cliques": lambda: (csr_from_dense(two_cliques(40)), 2),
        "tiny": lambda: (gen.grid(1, 3), 8),
        "isolated": lambda: (gen.random_graph(500, 1.0, 32, isolated_frac=0.6), 4),
        "path": lambda: (gen.grid(1, 300), 3),
    }[name]()
    _rounds(kmp, g, k, 2, 8, 2, name)


@pytest.mark.parametrize("name,k,passes", [
    ("grid128", 8, 2), ("rgg20000", 64, 2), ("rgg20000", 12, 5), ("rand_w", 7, 2), ("rand_iso", 16, 1),
])
def test_partition_fm(kmp, name, k, passes):
    g = {
        "grid128": lambda: gen.grid(128, 128),
        "rgg20000": lambda: gen.rgg(20000, 8.0, 2),
        "rand_w": lambda: gen.random_graph(5000, 5.0, 7, max_vw=4, max_ew=6),
        "rand_iso": lambda: gen.random_graph(8000, 3.0, 8, isolated_frac=0.3),
    }[name]()
    say(f"[fm partition] {name} k={k} passes={passes}")
    ref = oracle.partition(g, k, 0.03, 1, fm_passes=passes)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, part, stats = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 1, fm_passes=passes)
    assert rc == ref.status
    assert np.array_equal(part.cpu().numpy(), ref.part)
    assert stats["cut"] == ref.stats["cut"]


def test_batch_fm_equals_single_calls(kmp):
    graphs = [(gen.grid(40, 40), 6), (gen.random_graph(3000, 5.0, 41, max_vw=3, max_ew=4), 9),
              (gen.rgg(5000, 8.0, 42), 16)]
    jobs = []
    for i, (g, k) in enumerate(graphs):
        xadj, adjncy, vwgt, adjwgt = dev(g)
        jobs.append(dict(xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, k=k, epsilon=0.03, seed=10 + i,
                         out=torch.empty(g.n, dtype=torch.int32, device="cuda")))
    say("[fm batch] 3 jobs passes=2")
    rc, res, _ = kmp.kmp_partition_batch(jobs, fm_passes=2)
    assert rc == 0
    for i, (g, k) in enumerate(graphs):
        ref = oracle.partition(g, k, 0.03, 10 + i, fm_passes=2)
        assert res[i]["status"] == ref.status
        assert np.array_equal(jobs[i]["out"].cpu().numpy(), ref.part)


def test_fm_pass_count_rejected(kmp):
    g = gen.grid(8, 8)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    for bad in (-1, 17):
        rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 4, 0.03, 1, fm_passes=bad)
        assert rc == kmp.KMP_EINVAL
        d_part = t32(np.zeros(g.n, np.int32))
        rc, _, _ = kmp.kmp_bipartition_round(xadj, adjncy, vwgt, adjwgt, 0, d_part, [0], [4], 20, 1, fm_passes=bad)
        assert rc == kmp.KMP_EINVAL


# ------------------------------------------------------------------ pool: BFS and random growths

@pytest.mark.parametrize("k,passes", [(2, 0), (16, 0), (16, 2), (5, 1)])
def test_bipartition_round_pool(kmp, k, passes):
    _rounds(kmp, gen.rgg(4000, 8.0, 21), k, 0, 3, passes, "rgg4000", pool=True)


@pytest.mark.parametrize("name", ["weighted", "heavy-lds-and-global", "dense-hybrid", "big-edge-weights", "heavy-30",
                                  "isolated", "path"])
def test_bipartition_pool_weighted_and_degenerate(kmp, name):
    g, k = {
        "weighted": lambda: (gen.random_graph(900, 5.0, 31, max_vw=20, max_ew=5), 7),
        "heavy-lds-and-global": lambda: (_heavy_nodes(3000, 35), 6),
        # many internal entries per block: keys in LDS, entries in global memory (then LDS as blocks shrink)
        "dense-hybrid": lambda: (gen.random_graph(1200, 48.0, 38, max_ew=3), 5),
        "big-edge-weights": lambda: (gen.random_graph(400, 5.0, 36, max_ew=300000), 4),
        # node weights up to 30
        "heavy-30": lambda: (gen.random_graph(600, 3.0, 37, max_vw=30, max_ew=3), 8),
        "isolated": lambda: (gen.random_graph(500, 1.0, 32, isolated_frac=0.6), 4),
        "path": lambda: (gen.grid(1, 300), 3),
    }[name]()
    for passes in (0, 2):
        _rounds(kmp, g, k, 2, 8, passes, name, pool=True)


@pytest.mark.parametrize("name,k,passes", [("grid128", 8, 0), ("rgg20000", 64, 0), ("rgg20000", 64, 2),
                                           ("rand_w", 7, 1)])
def test_partition_pool(kmp, name, k, passes):
    g = {
        "grid128": lambda: gen.grid(128, 128),
        "rgg20000": lambda: gen.rgg(20000, 8.0, 2),
        "rand_w": lambda: gen.random_graph(5000, 5.0, 7, max_vw=4, max_ew=6),
    }[name]()
    say(f"[pool partition] {name} k={k} passes={passes}")
    ref = oracle.partition(g, k, 0.03, 1, fm_passes=passes, pool=True)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, part, stats = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 1, fm_passes=passes, ip_pool=True)
    assert rc == ref.status
    assert np.array_equal(part.cpu().numpy(), ref.part)
    assert stats["cut"] == ref.stats["cut"]


def test_batch_pool_equals_oracle(kmp):
    graphs = [(gen.grid(40, 40), 6), (gen.random_graph(3000, 5.0, 41, max_vw=3, max_ew=4), 9)]
    jobs = []
    for i, (g, k) in enumerate(graphs):
        xadj, adjncy, vwgt, adjwgt = dev(g)
        jobs.append(dict(xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, k=k, epsilon=0.03, seed=20 + i,
                         out=torch.empty(g.n, dtype=torch.int32, device="cuda")))
    say("[pool batch] 2 jobs passes=1")
    rc, res, _ = kmp.kmp_partition_batch(jobs, fm_passes=1, ip_pool=True)
    assert rc == 0
    for i, (g, k) in enumerate(graphs):
        ref = oracle.partition(g, k, 0.03, 20 + i, fm_passes=1, pool=True)
        assert res[i]["status"] == ref.status
        assert np.array_equal(jobs[i]["out"].cpu().numpy(), ref.part)


def test_pool_flag_rejected(kmp):
    g = gen.grid(8, 8)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 4, 0.03, 1, ip_pool=2)
    assert rc == kmp.KMP_EINVAL
    d_part = t32(np.zeros(g.n, np.int32))
    rc, _, _ = kmp.kmp_bipartition_round(xadj, adjncy, vwgt, adjwgt, 0, d_part, [0], [4], 20, 1, ip_pool=2)
    assert rc == kmp.KMP_EINVAL


# ------------------------------------------------------------------ adaptive imbalance of the bipartitions

@pytest.mark.parametrize("name,k,passes,pool", [
    ("grid128", 8, 0, False), ("rgg20000", 64, 0, False), ("rgg20000", 12, 2, False), ("rand_w", 7, 0, False),
    ("rand_w", 7, 1, True), ("rand_iso", 16, 0, False), ("rmat13", 100, 0, False), ("heavy3000", 6, 2, True),
])
def test_partition_adaptive_eps(kmp, name, k, passes, pool):
    g = {
        "grid128": lambda: gen.grid(128, 128),
        "rgg20000": lambda: gen.rgg(20000, 8.0, 2),
        "rand_w": lambda: gen.random_graph(5000, 5.0, 7, max_vw=4, max_ew=6),
        "rand_iso": lambda: gen.random_graph(8000, 3.0, 8, isolated_frac=0.3),
        "rmat13": lambda: gen.rmat(13, 8 << 13, seed=4),
        "heavy3000": lambda: _heavy_nodes(3000, 35),
    }[name]()
    say(f"[adaptive eps partition] {name} k={k} passes={passes} pool={pool}")
    ref = oracle.partition(g, k, 0.03, 1, fm_passes=passes, pool=pool, adaptive_eps=True)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, part, stats = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 1, fm_passes=passes,
                                           ip_pool=pool, adaptive_eps=True)
    assert rc == ref.status
    assert np.array_equal(part.cpu().numpy(), ref.part)
    assert stats["cut"] == ref.stats["cut"]


def test_batch_adaptive_eps_equals_oracle(kmp):
    specs = [(gen.grid(40, 60), 5, 1), (gen.rgg(3000, 8.0, 5), 16, 2), (gen.random_graph(2500, 4.0, 6, max_vw=3), 9, 3)]
    jobs = []
    for g, k, seed in specs:
        xadj, adjncy, vwgt, adjwgt = dev(g)
        jobs.append(dict(xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, k=k, epsilon=0.03, seed=seed,
                         out=torch.empty(g.n, dtype=torch.int32, device="cuda")))
    say("[adaptive eps batch] 3 jobs")
    rc, res, _ = kmp.kmp_partition_batch(jobs, adaptive_eps=True)
    assert rc == 0
    for (g, k, seed), j, r in zip(specs, jobs, res):
        ref = oracle.partition(g, k, 0.03, seed, adaptive_eps=True)
        assert r["status"] == ref.status and r["cut"] == ref.stats["cut"]
        assert np.array_equal(j["out"].cpu().numpy(), ref.part)


def test_adaptive_eps_flag_rejected(kmp):
    g = gen.grid(10, 10)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 4, 0.03, 1, adaptive_eps=2)
    assert rc == kmp.KMP_EINVAL
