"""GPU: the asynchronous LP mode (paper Sec. 5.1 "Parallelization" and
"Iteration Order", Sec. 5.3 "Local Improvement").

A parallel asynchronous run has no unique result, so it is checked two ways:

* executed one node per launch in visit order (serial = 1, async_lp = 2) the
  kernels are the one-processing-element execution, which must equal the
  oracle's sequential reading (O3b) bit for bit: single LP calls of both
  kinds over every rating tier (lane, LDS, hubs), whole partitions and a
  batch;
* in parallel (async_lp = 1) every result must be valid: labels in range,
  weights equal to the label sums, refinement within its bounds, partitions
  balanced, and the cut close to the deterministic mode's.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.helpers import node_w, with_hubs

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


def t64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).cuda()


def _lp_graphs():
    """Every rating tier: degrees < 16 (lane), < 64 and < 4096 (LDS tables), >= 4096 (hubs)."""
    return [("grid30x40", gen.grid(30, 40)),
            ("rgg3000", gen.rgg(3000, 8.0, seed=4)),
            ("weighted2500", gen.random_graph(2500, 6.0, 8, max_vw=4, max_ew=9)),
            ("rmat12", gen.rmat(12, 8 << 12, seed=5)),
            ("rgg6000+hubs", with_hubs(gen.rgg(6000, 6.0, 7), [4100, 5000], seed=3))]


@pytest.mark.parametrize("gi", range(5))
def test_lp_async_serial_cluster_matches_oracle(kmp, gi):
    name, g = _lp_graphs()[gi]
    c = node_w(g)
    for U, level, seed in ((5, 0, 3), (int(c.sum() // 50) + 1, 2, 11)):
        say(f"[lp_async serial cluster] {name} maxdeg={int(np.diff(g.xadj).max())} U={U}")
        n = g.n
        exp_label, exp_cw, exp_fav, exp_moves, exp_rounds = oracle.lp_async(
            g, level, oracle.T_CL, seed, np.arange(n, dtype=np.int32), c, caps=U, fav=np.zeros(n, np.uint32))
        xadj, adjncy, vwgt, adjwgt = dev(g)
        label = t32(np.arange(n))
        cw = t64(c)
        fav = torch.zeros(n, dtype=torch.int32, device="cuda")
        r, moves = kmp.kmp_lp_async(xadj, adjncy, vwgt, adjwgt, level, oracle.T_CL, seed, label, cw,
                                    cap_scalar=U, fav=fav, serial=True)
        assert r == exp_rounds and moves == list(exp_moves), name
        assert np.array_equal(label.cpu().numpy(), exp_label), name
        assert np.array_equal(cw.cpu().numpy(), exp_cw), name
        assert np.array_equal(fav.cpu().numpy().view(np.uint32), exp_fav), name


@pytest.mark.parametrize("gi", range(5))
def test_lp_async_serial_refine_matches_oracle(kmp, gi):
    name, g = _lp_graphs()[gi]
    c = node_w(g)
    rng = np.random.default_rng(gi)
    for nb, level, seed in ((4, 1, 5), (37, 0, 8)):
        say(f"[lp_async serial refine] {name} nb={nb}")
        part = rng.integers(0, nb, g.n).astype(np.int32)
        wt = np.bincount(part, weights=c, minlength=nb).astype(np.int64)
        cap = wt + rng.integers(0, max(2, int(c.sum() // (20 * nb))), nb)
        exp_part, exp_wt, _, exp_moves, exp_rounds = oracle.lp_async(g, level, oracle.T_REF, seed, part, wt,
                                                                     capv=cap)
        xadj, adjncy, vwgt, adjwgt = dev(g)
        d_part, d_wt = t32(part), t64(wt)
        r, moves = kmp.kmp_lp_async(xadj, adjncy, vwgt, adjwgt, level, oracle.T_REF, seed, d_part, d_wt,
                                    cap_vec=t64(cap), serial=True)
        assert r == exp_rounds and moves == list(exp_moves), name
        assert np.array_equal(d_part.cpu().numpy(), exp_part), name
        assert np.array_equal(d_wt.cpu().numpy(), exp_wt), name


def _partition_cases():
    return [("grid40x50", gen.grid(40, 50), 8),
            ("rgg3000", gen.rgg(3000, 8.0, seed=3), 16),
            ("weighted2000", gen.random_graph(2000, 5.0, 12, max_vw=5, max_ew=7), 7),
            ("rmat12", gen.rmat(12, 8 << 12, seed=9), 64)]


@pytest.mark.parametrize("ci", range(4))
def test_partition_async_serial_matches_oracle(kmp, ci):
    name, g, k = _partition_cases()[ci]
    say(f"[partition async serial] {name} k={k}")
    ref = oracle.partition(g, k, 0.03, 5, async_lp=True)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, out, st = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 5, async_lp=2)
    assert rc == ref.status, name
    assert np.array_equal(out.cpu().numpy(), ref.part), name
    assert st["cut"] == ref.stats["cut"] and st["level_n"] == ref.stats["level_n"], name
    assert st["lp_cluster_moves"] == ref.stats["lp_cluster_moves"], name
    assert st["lp_refine_moves"] == ref.stats["lp_refine_moves"], name


def test_batch_async_serial_matches_oracle(kmp):
    cases = _partition_cases()
    jobs = []
    for name, g, k in cases:
        xadj, adjncy, vwgt, adjwgt = dev(g)
        jobs.append(dict(xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, k=k, epsilon=0.03, seed=2,
                         out=torch.full((g.n,), -5, dtype=torch.int32, device="cuda")))
    say(f"[batch async serial] {len(jobs)} jobs")
    rc, res, _ = kmp.kmp_partition_batch(jobs, async_lp=2)
    assert rc >= 0
    for (name, g, k), j, r in zip(cases, jobs, res):
        ref = oracle.partition(g, k, 0.03, 2, async_lp=True)
        assert r["status"] == ref.status, name
        assert np.array_equal(j["out"].cpu().numpy(), ref.part), name
        assert r["cut"] == ref.stats["cut"], name


@pytest.mark.parametrize("name", ["rgg65536", "rmat16", "weighted50000"])
def test_lp_async_parallel_valid(kmp, name):
    g = {"rgg65536": lambda: gen.rgg(65536, 8.0, seed=2),
         "rmat16": lambda: gen.rmat(16, 8 << 16, seed=3),
         "weighted50000": lambda: gen.random_graph(50000, 7.0, 5, max_vw=4, max_ew=9)}[name]()
    c = node_w(g)
    n = g.n
    xadj, adjncy, vwgt, adjwgt = dev(g)
    U = int(c.sum() // 2000) + int(c.max())
    say(f"[lp_async parallel cluster] {name} U={U}")
    label, cw = t32(np.arange(n)), t64(c)
    fav = torch.zeros(n, dtype=torch.int32, device="cuda")
    r, moves = kmp.kmp_lp_async(xadj, adjncy, vwgt, adjwgt, 0, oracle.T_CL, 7, label, cw, cap_scalar=U, fav=fav)
    lab, w = label.cpu().numpy(), cw.cpu().numpy()
    assert 1 <= r <= oracle.ROUNDS and moves[0] > 0 and all(m >= 0 for m in moves)
    assert lab.min() >= 0 and lab.max() < n
    assert np.array_equal(w, np.bincount(lab, weights=c, minlength=n).astype(np.int64))
    nc = len(np.unique(lab))
    say(f"  clusters {nc} of {n}, moves {moves}, largest {w.max()} (U {U})")
    assert nc < 0.7 * n
    # refinement: the bounds hold strictly, weights follow the labels
    nb = 64
    rng = np.random.default_rng(1)
    part = rng.integers(0, nb, n).astype(np.int32)
    wt = np.bincount(part, weights=c, minlength=nb).astype(np.int64)
    cap = wt + int(c.sum() // (nb * 50)) + 1
    say(f"[lp_async parallel refine] {name} nb={nb}")
    d_part, d_wt = t32(part), t64(wt)
    r, moves = kmp.kmp_lp_async(xadj, adjncy, vwgt, adjwgt, 0, oracle.T_REF, 9, d_part, d_wt, cap_vec=t64(cap))
    p, w = d_part.cpu().numpy(), d_wt.cpu().numpy()
    assert 1 <= r <= oracle.ROUNDS and moves[0] > 0
    assert p.min() >= 0 and p.max() < nb
    assert np.array_equal(w, np.bincount(p, weights=c, minlength=nb).astype(np.int64))
    assert (w <= cap).all()
    A_cut_before = oracle.cut(g, part)
    assert oracle.cut(g, p) < A_cut_before


@pytest.mark.parametrize("name", ["grid60", "rgg5000", "weighted4000"])
def test_lp_async_small_level_valid(kmp, name):
    """Levels of at most 8192 nodes run the asynchronous call in one workgroup (LDS labels and weights):
    the same validity checks as the launch path."""
    g = {"grid60": lambda: gen.grid(60, 60), "rgg5000": lambda: gen.rgg(5000, 8.0, seed=6),
         "weighted4000": lambda: gen.random_graph(4000, 6.0, 3, max_vw=4, max_ew=9)}[name]()
    c = node_w(g)
    n = g.n
    xadj, adjncy, vwgt, adjwgt = dev(g)
    U = int(c.sum() // 300) + int(c.max())
    say(f"[lp_async small cluster] {name} U={U}")
    label, cw = t32(np.arange(n)), t64(c)
    r, moves = kmp.kmp_lp_async(xadj, adjncy, vwgt, adjwgt, 1, oracle.T_CL, 3, label, cw, cap_scalar=U)
    lab, w = label.cpu().numpy(), cw.cpu().numpy()
    assert 1 <= r <= oracle.ROUNDS and moves[0] > 0
    assert lab.min() >= 0 and lab.max() < n
    assert np.array_equal(w, np.bincount(lab, weights=c, minlength=n).astype(np.int64))
    assert len(np.unique(lab)) < 0.7 * n
    nb = 16
    rng = np.random.default_rng(2)
    part = rng.integers(0, nb, n).astype(np.int32)
    wt = np.bincount(part, weights=c, minlength=nb).astype(np.int64)
    cap = wt + int(c.sum() // (nb * 40)) + 1
    say(f"[lp_async small refine] {name} nb={nb}")
    d_part, d_wt = t32(part), t64(wt)
    r, moves = kmp.kmp_lp_async(xadj, adjncy, vwgt, adjwgt, 1, oracle.T_REF, 4, d_part, d_wt, cap_vec=t64(cap))
    p, w = d_part.cpu().numpy(), d_wt.cpu().numpy()
    assert 1 <= r <= oracle.ROUNDS and moves[0] > 0
    assert np.array_equal(w, np.bincount(p, weights=c, minlength=nb).astype(np.int64))
    assert (w <= cap).all()
    assert oracle.cut(g, p) < oracle.cut(g, part)


@pytest.mark.parametrize("name,k", [("rgg65536", 64), ("grid128", 8), ("rmat16", 256), ("weighted50000", 31)])
def test_partition_async_parallel_valid(kmp, name, k):
    g = {"rgg65536": lambda: gen.rgg(65536, 8.0, seed=2), "grid128": lambda: gen.grid(128, 128),
         "rmat16": lambda: gen.rmat(16, 8 << 16, seed=3),
         "weighted50000": lambda: gen.random_graph(50000, 7.0, 5, max_vw=4, max_ew=9)}[name]()
    xadj, adjncy, vwgt, adjwgt = dev(g)
    say(f"[partition async parallel] {name} k={k}")
    rc_d, out_d, st_d = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 1)
    rc, out, st = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 1, async_lp=1)
    p = out.cpu().numpy()
    c = node_w(g)
    bw = np.bincount(p, weights=c, minlength=k)
    say(f"  cut async {st['cut']} deterministic {st_d['cut']}, max block {int(bw.max())} (L_k {st['lk']})")
    assert rc == rc_d == kmp.KMP_OK
    assert p.min() >= 0 and p.max() < k
    assert int(bw.max()) == st["max_block_weight"] <= st["lk"]
    assert st["cut"] == oracle.cut(g, p)
    assert st["cut"] <= 1.25 * st_d["cut"] + 10


def test_async_options_rejected(kmp):
    g = gen.grid(10, 10)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 4, 0.03, 1, async_lp=3)
    assert rc == kmp.KMP_EINVAL
    label, cw = t32(np.arange(g.n)), t64(np.ones(g.n))
    r, _ = kmp.kmp_lp_async(xadj, adjncy, vwgt, adjwgt, 0, 4, 1, label, cw, cap_scalar=3)
    assert r == kmp.KMP_EINVAL
