"""Pins of the oracle's asynchronous LP (O3b), restated here from the paper
(dense matrices and plain Python, no oracle code path) and compared with the
oracle exactly.

Sec. 5.1 "Parallelization": the asynchronous mode updates cluster weights at
once, so a node visited later sees every earlier move.  Sec. 5.1 "Iteration
Order": nodes are visited by exponentially spaced degree buckets
(2^i <= d < 2^(i+1)), split into chunks traversed in random order; the
reading takes the hash classes of the sub-round LP as those chunks, class
by class.  Executed by one processing element this is a sequential LP:
visits in ascending (class, bucket, id), each against the current state,
with the rounds, early exit and active rule of the deterministic LP
(Sec. 5.1 Coarsening, Sec. 5.3 Local Improvement).

Each test also checks that its cases exercise the rule: immediate updates
change the result against rating a round's nodes on its start state, the
bucket order and the class order each change it, and later rounds move.
"""
import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.helpers import dense_adj, node_w


def _bucket(d):
    return 0 if d <= 1 else int(d).bit_length() - 1


def _visit_order(g, seed, level, classes=True, buckets=True):
    deg = np.diff(np.asarray(g.xadj, np.int64))
    return sorted(range(g.n), key=lambda v: (oracle.sub_class(seed, level, v) if classes else 0,
                                             _bucket(int(deg[v])) if buckets else 0, v))


def _rate_one(A, label, v, nlab):
    r = np.zeros(nlab, np.int64)
    for u in np.nonzero(A[v])[0]:
        r[label[u]] += A[v, u]
    return r


def _async_call(g, level, tag, seed, label, wt, cap, order=None, immediate=True):
    """Sequential LP: every active node in `order`, rated against the current state (immediate=True) or
    against the state at the round's start (immediate=False, for the coverage check only)."""
    A = dense_adj(g)
    c = node_w(g)
    n = g.n
    nlab = wt.shape[0]
    order = _visit_order(g, seed, level) if order is None else order
    label, wt = label.copy(), wt.copy()
    fav = {}
    active = np.ones(n, bool)
    moves = []
    for r in range(oracle.ROUNDS):
        moved = np.zeros(n, bool)
        start_label, start_wt = label.copy(), wt.copy()
        for v in order:
            if not active[v]:
                continue
            see_l, see_w = (label, wt) if immediate else (start_label, start_wt)
            R = _rate_one(A, see_l, v, nlab)
            own = int(see_l[v])
            ks = [K for K in range(nlab) if K != own and R[K] > 0]
            ks.sort(key=lambda K: (-int(R[K]), oracle.hash_(seed, tag, level, r, K), K))
            fav[v] = ks[0] if ks else oracle.NONE
            fits = [K for K in ks if see_w[K] + c[v] <= cap[K]]
            if fits and R[fits[0]] > R[own]:
                K = fits[0]
                wt[K] += c[v]
                wt[label[v]] -= c[v]
                label[v] = K
                moved[v] = True
        moves.append(int(moved.sum()))
        if not moved.any():
            break
        active = (A[:, moved] > 0).any(axis=1)
    return label, wt, fav, moves


def _cases():
    out = []
    for seed in range(40):
        n = 9 + seed % 6
        g = gen.random_graph(n, 2.5 + (seed % 4), 4100 + seed, max_vw=3, max_ew=5)
        out.append((seed, g))
    return out


@pytest.mark.parametrize("tag", ["cluster", "refine"])
def test_async_lp_restated_visit_by_visit(tag):
    later_rounds = 0  # cases whose later rounds moved something
    sees_moves = 0    # cases where seeing earlier moves at once changed the result
    bucket_order = 0  # cases where the degree-bucket order changed the result against id order
    class_order = 0   # cases where the class order changed the result against bucket order alone
    for seed, g in _cases():
        n = g.n
        c = node_w(g)
        rng = np.random.default_rng(seed)
        level, hseed = int(rng.integers(0, 6)), int(rng.integers(1, 2**40))
        if tag == "cluster":
            label = np.arange(n, dtype=np.int32)
            wt = c.copy()
            U = int(rng.integers(3, 8))
            cap = np.full(n, U, np.int64)
            t = oracle.T_CL
            got = oracle.lp_async(g, level, t, hseed, label, wt, caps=U, fav=np.zeros(n, np.uint32))
        else:
            nb = 3
            label = rng.integers(0, nb, n).astype(np.int32)
            wt = np.bincount(label, weights=c, minlength=nb).astype(np.int64)
            cap = wt + rng.integers(0, 6, nb)
            t = oracle.T_REF
            got = oracle.lp_async(g, level, t, hseed, label, wt, capv=cap)
        exp_label, exp_wt, exp_fav, exp_moves = _async_call(g, level, t, hseed, label, wt, cap)
        g_label, g_wt, g_fav, g_moves, g_rounds = got
        assert np.array_equal(g_label, exp_label), seed
        assert np.array_equal(g_wt, exp_wt), seed
        assert list(g_moves[:len(exp_moves)]) == exp_moves, seed
        assert (np.asarray(g_moves[len(exp_moves):]) == 0).all(), seed
        assert g_rounds == len(exp_moves), seed
        if tag == "cluster":
            for v in range(n):
                assert int(g_fav[v]) == int(exp_fav.get(v, 0)), (seed, v)
        # the bound holds strictly for a single processing element
        assert (exp_wt <= np.maximum(cap[:len(exp_wt)], wt)).all()
        later_rounds += any(m > 0 for m in exp_moves[1:])
        jac = _async_call(g, level, t, hseed, label, wt, cap, immediate=False)
        sees_moves += not np.array_equal(jac[0], exp_label)
        ids = _async_call(g, level, t, hseed, label, wt, cap, order=_visit_order(g, hseed, level, buckets=False))
        bucket_order += not np.array_equal(ids[0], exp_label)
        nocl = _async_call(g, level, t, hseed, label, wt, cap, order=_visit_order(g, hseed, level, classes=False))
        class_order += not np.array_equal(nocl[0], exp_label)
    assert later_rounds >= 5
    assert sees_moves >= 10
    assert bucket_order >= 5
    assert class_order >= 5


def test_async_lp_weights_follow_labels_and_clusters_respect_bound():
    """Invariants on larger graphs: the weights are the label sums and no cluster exceeds U."""
    for seed, (n, d) in enumerate([(300, 6.0), (500, 9.0), (800, 4.0)]):
        g = gen.random_graph(n, d, 77 + seed, max_vw=4, max_ew=7)
        c = node_w(g)
        U = int(c.sum() // 40)
        lab, cw, fav, moves, rounds = oracle.lp_async(g, 2, oracle.T_CL, 5 + seed, np.arange(n, dtype=np.int32),
                                                     c.copy(), caps=U, fav=np.zeros(n, np.uint32))
        assert np.array_equal(cw, np.bincount(lab, weights=c, minlength=n).astype(np.int64))
        assert (cw <= np.maximum(U, c)).all()
        assert moves[0] > 0 and 1 <= rounds <= oracle.ROUNDS
        assert len(np.unique(lab)) < n


def test_partition_with_async_lp_differs_and_stays_valid():
    """The option reaches every LP call: the partition changes, stays balanced, and the cut stays close to
    the deterministic one on these graphs."""
    differ = 0
    for g, k in [(gen.grid(40, 50), 8), (gen.rgg(3000, 8.0, seed=3), 16), (gen.grid(64, 64), 4)]:
        a = oracle.partition(g, k, 0.03, 1, async_lp=True)
        d = oracle.partition(g, k, 0.03, 1)
        assert a.status == oracle.OK and d.status == oracle.OK
        assert a.stats["max_block_weight"] <= a.stats["lk"]
        assert a.part.min() >= 0 and a.part.max() < k and len(np.unique(a.part)) == k
        differ += not np.array_equal(a.part, d.part)
        assert a.stats["cut"] <= 1.5 * d.stats["cut"]
    assert differ >= 2
