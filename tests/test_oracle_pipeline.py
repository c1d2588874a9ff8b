"""Whole-pipeline pins of the oracle: brute force, special cases, invariants."""
import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.helpers import brute_force_min_cut, csr_from_dense, cut_dense, dense_adj, node_w, path, two_cliques


def _check_result(g, k, eps, res):
    n = g.n
    c = node_w(g)
    assert res.part.shape == (n,)
    if n:
        assert res.part.min() >= 0 and res.part.max() < k
    bw = np.bincount(res.part, weights=c, minlength=k)
    lk = oracle.lk(int(c.sum()), k, eps)
    assert res.stats["lk"] == lk if k > 1 or n else True
    if res.status == oracle.OK:
        assert bw.max() <= lk
    else:
        assert res.status == oracle.IMBALANCED and bw.max() > lk
    assert res.stats["cut"] == cut_dense(dense_adj(g), res.part) if n <= 400 else True
    return bw, lk


@pytest.mark.parametrize("seed", range(10))
def test_brute_force_small(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 9))
    k = int(rng.integers(2, 4))
    g = gen.random_graph(n, 3.0, seed, max_ew=4)
    A = dense_adj(g)
    c = node_w(g)
    res = oracle.partition(g, k, 0.03, seed)
    bw, lk = _check_result(g, k, 0.03, res)
    opt = brute_force_min_cut(A, c, k, lk)
    assert res.status == oracle.OK            # unit weights: always repairable
    assert res.stats["cut"] >= opt


def test_two_cliques_k2_cut_zero():
    for s in (20, 60, 150):
        g = csr_from_dense(two_cliques(s))
        res = oracle.partition(g, 2, 0.03, 1)
        assert res.status == oracle.OK
        assert res.stats["cut"] == 0
        assert np.bincount(res.part).tolist() == [s, s]


def test_k1_all_zero():
    g = gen.grid(10, 10)
    res = oracle.partition(g, 1, 0.03, 1)
    assert res.status == oracle.OK and (res.part == 0).all()


def test_empty_graph():
    g = gen.Graph(np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert oracle.partition(g, 4, 0.03, 1).status == oracle.OK


def test_k_larger_than_n_allows_empty_blocks():
    g = gen.grid(2, 3)
    res = oracle.partition(g, 16, 0.03, 1)
    assert res.status == oracle.OK
    assert np.bincount(res.part, minlength=16).max() <= 1


def test_eps_zero_and_isolated_nodes():
    g = gen.random_graph(500, 2.0, 9, isolated_frac=0.3)
    for eps in (0.0, 0.03):
        res = oracle.partition(g, 5, eps, 3)
        _check_result(g, 5, eps, res)
        assert res.status == oracle.OK


def test_single_edge():
    g = csr_from_dense(path(2))
    res = oracle.partition(g, 2, 0.03, 1)
    assert sorted(res.part.tolist()) == [0, 1] and res.stats["cut"] == 1


def test_deterministic():
    g = gen.rgg(5000, 8.0, 3)
    a = oracle.partition(g, 12, 0.03, 5)
    b = oracle.partition(g, 12, 0.03, 5)
    assert np.array_equal(a.part, b.part)
    c = oracle.partition(g, 12, 0.03, 6)
    assert not np.array_equal(a.part, c.part)   # the seed matters


@pytest.mark.parametrize("name,k", [("grid", 8), ("rgg", 12), ("rgg", 64), ("rand", 7)])
def test_invariants_through_trace(name, k):
    if name == "grid":
        g = gen.grid(64, 64)
    elif name == "rgg":
        g = gen.rgg(20000, 8.0, 2)
    else:
        g = gen.random_graph(6000, 4.0, 4, max_vw=3, max_ew=5, isolated_frac=0.05)
    res = oracle.partition(g, k, 0.03, 1, trace=True)
    assert res.status == oracle.OK
    tr = res.trace
    L = res.stats["levels"]
    levels = [g]
    for l in range(L):
        cg = gen.Graph(tr[("coarse_xadj", l + 1)], tr[("coarse_adjncy", l + 1)], tr[("coarse_vwgt", l + 1)],
                       tr[("coarse_adjwgt", l + 1)])
        levels.append(cg)
        # contraction conserves node weight; shrinks
        assert int(np.sum(cg.vwgt)) == int(node_w(g).sum())
        assert cg.n < levels[l].n
        # every cluster of level l respects U_l (unit input weights => U_l caps coarse node weights)
    for l in range(L, -1, -1):
        gl = levels[l]
        part = tr[("refine", l)]
        first, fc = tr[("first", l)], tr[("fcount", l)]
        nb = len(first)
        assert int(fc.sum()) == k                       # sum of final block counts
        assert (np.diff(first) > 0).all() and first[0] == 0
        # invariant (P): number of blocks after the bipartition loop
        kp = k if l == 0 else min(k, 1 << int(np.ceil(np.log2(max(1.0, gl.n / 160)))))
        kp = max(kp, 2)
        assert nb >= kp and nb < 2 * kp
        # invariant (B) after balancing: blocks within f_B * L_k (unit node weights at level 0)
        lk = res.stats["lk"]
        bw = np.bincount(tr[("balance", l)], weights=node_w(gl), minlength=nb)
        if l == 0:
            assert (bw <= fc * lk).all()
        # refinement keeps caps and never increases the cut
        bwr = np.bincount(part, weights=node_w(gl), minlength=nb)
        assert (bwr <= np.maximum(fc * lk, bw)).all()
        assert oracle.cut(gl, part) <= oracle.cut(gl, tr[("balance", l)])
        if l < L:
            # projection keeps the cut and the block weights
            mp = tr[("map", l)]
            proj = tr[("project", l)]
            coarse_part = tr[("refine", l + 1)]
            assert np.array_equal(proj, coarse_part[mp])
            assert oracle.cut(gl, proj) == oracle.cut(levels[l + 1], coarse_part)


def test_errors():
    g = gen.grid(4, 4)
    assert oracle.partition(g, 0, 0.03, 1).status == oracle.EINVAL
    assert oracle.partition(g, 2, -0.1, 1).status == oracle.EINVAL
    assert oracle.partition(g, 2, float("nan"), 1).status == oracle.EINVAL
    bad = gen.Graph(g.xadj.copy(), g.adjncy.copy())
    bad.adjncy[0] = 5                                   # asymmetric
    assert oracle.partition(bad, 2, 0.03, 1).status == oracle.EGRAPH
    loop = gen.Graph(np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32))
    assert oracle.partition(loop, 2, 0.03, 1).status == oracle.EGRAPH
    dup = gen.Graph(np.array([0, 2, 4], np.int32), np.array([1, 1, 0, 0], np.int32))
    assert oracle.partition(dup, 2, 0.03, 1).status == oracle.EGRAPH
    neg = gen.Graph(g.xadj.copy(), g.adjncy.copy(), vwgt=np.zeros(16, np.int32))
    assert oracle.partition(neg, 2, 0.03, 1).status == oracle.EGRAPH
    big = gen.Graph(g.xadj.copy(), g.adjncy.copy(), vwgt=np.full(16, 2**28, np.int32))
    assert oracle.partition(big, 2, 0.03, 1).status == oracle.EOVERFLOW


def test_weighted_imbalanced_status():
    # one node heavier than L_k: no partition can be balanced -> status 1
    A = path(6)
    g = csr_from_dense(A, vwgt=[1, 1, 1, 1, 1, 20])
    res = oracle.partition(g, 3, 0.03, 1)
    assert res.status == oracle.IMBALANCED


def test_grid_quality_reference_layout():
    # 128x128, k=8: a 2x4 rectangle layout cuts 512 edges; report, do not pin quality
    g = gen.grid(128, 128)
    res = oracle.partition(g, 8, 0.03, 1)
    assert res.status == oracle.OK
    assert res.stats["cut"] < 3 * 512
