"""Pins of the oracle's multi-step rules, each restated here from the reading
of the paper it follows (dense matrices and plain Python, no oracle code
path), and compared with the oracle's own result exactly.

* a whole LP call: sub-rounds of hash classes, the active set of a round
  (nodes with a neighbour that moved in the previous round), the stop after
  a round without moves and the cap of 5 rounds (Sec. 5.1 Coarsening,
  Sec. 5.3 Local Improvement)
* one bipartitionBlocks round (Alg. 2; Sec. 4 Handling General k): block
  extraction with ranks as local ids and internal edges only, the split of
  f into floor(f/2) and ceil(f/2), renumbering by first
* the exact two-hop pair list (Sec. 5.1 Two-hop Clustering)
* the balancer's rounds with several overloaded blocks competing for one
  target, and the most-free-block fallback (Sec. 5.3 Balancing)

Each test also checks that its case exercises the rule it pins (a round
after the first moved something, the limit bound, a target was contended),
so that a plausible slip in the rule changes the expected result.
"""
import fractions

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.helpers import dense_adj, indicator, node_w


# ---------------------------------------------------------------- LP call

def _rate(A, label, nlab):
    return A @ indicator(label, nlab)


def _subround(A, c, label, wt, cap, members, seed, tag, level, r, want_fav):
    """One sub-round: every member is rated against the state at the sub-round's start, then admission
    per target in ascending node id (longest fitting prefix), then apply."""
    nlab = wt.shape[0]
    R = _rate(A, label, nlab)
    props, fav = [], {}
    for v in members:
        own = int(label[v])
        ks = [K for K in range(nlab) if K != own and R[v, K] > 0]
        ks.sort(key=lambda K: (-int(R[v, K]), oracle.hash_(seed, tag, level, r, K), K))
        if want_fav:
            fav[v] = ks[0] if ks else oracle.NONE
        fits = [K for K in ks if wt[K] + c[v] <= cap[K]]
        if fits and R[v, fits[0]] > R[v, own]:
            props.append((fits[0], v))
    props.sort()
    new_label, new_wt = label.copy(), wt.copy()
    moved = []
    run = {}
    for K, v in props:
        run[K] = run.get(K, 0) + int(c[v])
        if wt[K] + run[K] <= cap[K]:
            new_wt[K] += c[v]
            new_wt[label[v]] -= c[v]
            new_label[v] = K
            moved.append(v)
    return new_label, new_wt, fav, moved


def _lp_call(g, level, tag, seed, label, wt, cap, want_fav):
    """A whole LP call: round 0 rates every node; round r+1 rates the nodes with a neighbour that moved in
    round r; a round without moves ends the call; at most 5 rounds.  Returns the state, the favoured
    clusters (last rating of each node), the moves per round and the number of rounds run."""
    A = dense_adj(g)
    c = node_w(g)
    n = g.n
    label, wt = label.copy(), wt.copy()
    fav = {}
    active = np.ones(n, bool)
    moves = []
    for r in range(oracle.ROUNDS):
        moved_r = np.zeros(n, bool)
        for s in range(4):
            members = [v for v in range(n) if active[v] and oracle.sub_class(seed, level, v) == s]
            label, wt, f, moved = _subround(A, c, label, wt, cap, members, seed, tag, level, r, want_fav)
            fav.update(f)
            moved_r[moved] = True
        moves.append(int(moved_r.sum()))
        if not moved_r.any():
            break
        active = (A[:, moved_r] > 0).any(axis=1)
    return label, wt, fav, moves


def _lp_cases():
    """Small graphs with tight cluster bounds, chosen so that LP runs several rounds."""
    out = []
    for seed in range(40):
        n = 8 + seed % 5
        g = gen.random_graph(n, 3.0 + (seed % 3), 900 + seed, max_vw=3, max_ew=5)
        out.append((seed, g))
    return out


@pytest.mark.parametrize("tag", ["cluster", "refine"])
def test_lp_call_restated_round_by_round(tag):
    multi_round = 0   # cases whose later rounds moved something
    restricted = 0    # cases where a later round's active set left out a node that still wanted to move
    for seed, g in _lp_cases():
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
            got = oracle.lp_generic(g, level, t, hseed, label, wt, caps=U, fav=np.zeros(n, np.uint32))
        else:
            nb = 3
            label = rng.integers(0, nb, n).astype(np.int32)
            wt = np.bincount(label, weights=c, minlength=nb).astype(np.int64)
            cap = wt + rng.integers(0, 6, nb)
            t = oracle.T_REF
            got = oracle.lp_generic(g, level, t, hseed, label, wt, capv=cap)
        exp_label, exp_wt, exp_fav, exp_moves = _lp_call(g, level, t, hseed, label, wt, cap, tag == "cluster")
        g_label, g_wt, g_fav, g_moves, g_rounds = got
        assert np.array_equal(g_label, exp_label), seed
        assert np.array_equal(g_wt, exp_wt), seed
        assert list(g_moves[:len(exp_moves)]) == exp_moves, seed
        assert (np.asarray(g_moves[len(exp_moves):]) == 0).all(), seed
        assert g_rounds == len(exp_moves), seed
        if tag == "cluster":
            for v in range(n):
                assert int(g_fav[v]) == int(exp_fav.get(v, 0)), (seed, v)
        multi_round += sum(1 for m in exp_moves[1:] if m > 0) > 0
        # would an unrestricted later round have moved a node outside the active set?
        if len(exp_moves) >= 2:
            A = dense_adj(g)
            lab1, wt1, _, _ = _lp_call(g, level, t, hseed, label, wt, cap, False)
            lab_all, _, _, mv = _subround(A, c, lab1, wt1, cap, list(range(n)), hseed, t, level, 9, False)
            restricted += len(mv) > 0
    assert multi_round >= 10
    assert restricted >= 1


def test_lp_call_five_round_cap_binds():
    """A case whose LP still moves in its fifth round: the cap, not convergence, ends it."""
    found = 0
    for seed in range(200):
        g = gen.random_graph(12, 4.0, 1200 + seed, max_vw=3, max_ew=6)
        n = g.n
        c = node_w(g)
        nb = 3
        rng = np.random.default_rng(seed)
        label = rng.integers(0, nb, n).astype(np.int32)
        wt = np.bincount(label, weights=c, minlength=nb).astype(np.int64)
        cap = wt + rng.integers(0, 4, nb)
        exp = _lp_call(g, 1, oracle.T_REF, 77 + seed, label, wt, cap, False)
        if len(exp[3]) == oracle.ROUNDS and exp[3][-1] > 0:
            got = oracle.lp_generic(g, 1, oracle.T_REF, 77 + seed, label, wt, capv=cap)
            assert np.array_equal(got[0], exp[0]) and list(got[3]) == exp[3] and got[4] == oracle.ROUNDS
            found += 1
            if found >= 3:
                break
    assert found >= 1


# ---------------------------------------------------------------- bipartition round

def _extract(g, part, b):
    """G[V_b]: the nodes of block b in ascending id, local id = rank, internal edges only (ascending)."""
    from paper_2105_02022_amd.gen import Graph
    nodes = np.nonzero(part == b)[0]
    local = {int(v): i for i, v in enumerate(nodes)}
    xadj, adj, ew = [0], [], []
    w = g.adjwgt if g.adjwgt is not None else np.ones(g.m, np.int32)
    for v in nodes:
        row = []
        for e in range(g.xadj[v], g.xadj[v + 1]):
            u = int(g.adjncy[e])
            if u in local:
                row.append((local[u], int(w[e])))
        row.sort()
        adj += [u for u, _ in row]
        ew += [x for _, x in row]
        xadj.append(len(adj))
    vw = None if g.vwgt is None else np.asarray(g.vwgt, np.int32)[nodes]
    sub = Graph(np.array(xadj, np.int32), np.array(adj, np.int32), vw,
                None if g.adjwgt is None else np.array(ew, np.int32), "sub")
    return nodes, sub


def _bip_round(g, level, part, first, f, lk_, seed):
    """Alg. 2 round: every block with f >= 2 becomes (first, floor(f/2)) [grown side 0] and
    (first + floor(f/2), ceil(f/2)) [side 1]; blocks with f = 1 stay; all blocks renumbered by first."""
    blocks = []       # (first, f, nodes assigned)
    for b in range(len(first)):
        nodes, sub = _extract(g, part, b)
        if f[b] < 2:
            blocks.append((first[b], f[b], nodes))
            continue
        side, _ = oracle.ggg(sub, level, first[b], f[b], lk_, seed)
        f0 = f[b] // 2
        blocks.append((first[b], f0, nodes[side == 0]))
        blocks.append((first[b] + f0, f[b] - f0, nodes[side == 1]))
    blocks.sort(key=lambda x: x[0])
    new = np.full(g.n, -1, np.int32)
    for i, (_, _, nodes) in enumerate(blocks):
        new[nodes] = i
    assert (new >= 0).all()
    return new, [x[0] for x in blocks], [x[1] for x in blocks]


@pytest.mark.parametrize("case", range(6))
def test_bipartition_round_restated(case):
    """Odd block counts (f = 3, 5, 7) so that floor/ceil matter; weighted nodes; a block of count 1
    that must be kept; several blocks, some not in ascending `first` order before renumbering."""
    rng = np.random.default_rng(40 + case)
    g = gen.random_graph(70 + 10 * case, 4.0, 40 + case, max_vw=3, max_ew=4)
    c = node_w(g)
    k = [7, 5, 11, 9, 13, 3][case]
    lk_ = oracle.lk(int(c.sum()), k, 0.03)
    part = np.zeros(g.n, np.int32)
    first, f = [0], [k]
    level = case
    seed = 500 + case
    rounds = 0
    while max(f) >= 2:
        exp_part, exp_first, exp_f = _bip_round(g, level, part, first, f, lk_, seed)
        got_part, got_first, got_f = oracle.bipartition_round(g, level, part, first, f, lk_, seed)
        assert list(got_first) == exp_first and list(got_f) == exp_f, (case, rounds)
        assert np.array_equal(got_part, exp_part), (case, rounds)
        part, first, f = exp_part, exp_first, exp_f
        rounds += 1
    assert sorted(first) == first and sum(f) == k and len(first) == k
    assert rounds == (k - 1).bit_length()


# ---------------------------------------------------------------- two-hop

def _two_hop(n, c, U, label, fav):
    """Singletons (labels with one member) sorted by (favoured cluster, id), NONE last; within a group
    positions (0,1), (2,3), ... form pairs; a pair is eligible if c(a) + c(b) <= U; the first
    min(#eligible, n_c - floor(n/2)) eligible pairs in that order merge b into a's cluster."""
    nc = len(np.unique(label))
    if nc <= n // 2:
        return label.copy(), []
    cnt = np.bincount(label, minlength=n)
    singles = sorted((int(fav[v]), v) for v in range(n) if cnt[label[v]] == 1)
    pairs = []
    i = 0
    while i < len(singles):
        j = i
        while j < len(singles) and singles[j][0] == singles[i][0]:
            j += 1
        for p in range(i, j - 1, 2):
            a, b = singles[p][1], singles[p + 1][1]
            if c[a] + c[b] <= U:
                pairs.append((a, b))
        i = j
    pairs = pairs[:nc - n // 2]
    new = label.copy()
    for a, b in pairs:
        new[b] = new[a]
    return new, pairs


@pytest.mark.parametrize("case", range(8))
def test_two_hop_exact_pairs(case):
    rng = np.random.default_rng(700 + case)
    n = 60 + 7 * case
    g = gen.random_graph(n, 3.0, 700 + case, max_vw=4)
    c = node_w(g)
    label = np.arange(n, dtype=np.int32)
    # some non-singleton clusters of q members; larger ones in later cases so the limit n_c - n/2 binds
    q = 2 + case % 4
    for v in range(0, q * (case + 2), q):
        label[v + 1:v + q] = label[v]
    cw = np.bincount(label, weights=c, minlength=n).astype(np.int64)
    fav = rng.integers(0, 4, n).astype(np.uint32)
    fav[rng.random(n) < 0.25] = oracle.NONE
    U = int(rng.integers(4, 8))
    exp, pairs = _two_hop(n, c, U, label, fav)
    got, got_cw, merged = oracle.two_hop(g, U, label, cw, fav)
    assert np.array_equal(got, exp), case
    assert merged == len(pairs)
    assert len(pairs) > 0
    assert np.array_equal(got_cw, np.bincount(exp, weights=c, minlength=n).astype(np.int64))


def test_two_hop_limit_binds_and_none_group_last():
    """The merge limit cuts the pair list, so the group order decides which pairs merge; isolated
    nodes (favoured cluster NONE) pair among themselves after every other group."""
    hits = 0
    for case in range(30):
        rng = np.random.default_rng(3000 + case)
        n = 40
        g = gen.random_graph(n, 2.0, 3000 + case)
        c = node_w(g)
        label = np.arange(n, dtype=np.int32)
        label[:15] = np.repeat(np.array([0, 5, 10], np.int32), 5)   # three clusters of five
        cw = np.bincount(label, weights=c, minlength=n).astype(np.int64)
        fav = rng.integers(0, 3, n).astype(np.uint32)
        fav[rng.random(n) < 0.4] = oracle.NONE
        exp, pairs = _two_hop(n, c, 10, label, fav)
        got = oracle.two_hop(g, 10, label, cw, fav)[0]
        assert np.array_equal(got, exp)
        every = _two_hop_all(n, c, 10, label, fav)
        left_out = every[len(pairs):]
        if left_out and any(fav[a] == oracle.NONE for a, _ in left_out):
            hits += 1
    assert hits >= 5


def _two_hop_all(n, c, U, label, fav):
    cnt = np.bincount(label, minlength=n)
    singles = sorted((int(fav[v]), v) for v in range(n) if cnt[label[v]] == 1)
    out = []
    i = 0
    while i < len(singles):
        j = i
        while j < len(singles) and singles[j][0] == singles[i][0]:
            j += 1
        for p in range(i, j - 1, 2):
            if c[singles[p][1]] + c[singles[p + 1][1]] <= U:
                out.append((singles[p][1], singles[p + 1][1]))
        i = j
    return out


# ---------------------------------------------------------------- balance

def _balance(g, level, seed, part, wt, cap):
    """Rounds while a block is overloaded and the previous round moved a node.  Per round: T* = the
    non-overloaded block with the most free room (smallest index on ties); every node of an overloaded
    block targets the most connected adjacent non-overloaded block it fits into (ties by the round's
    hash, then index), else T* if it fits; candidates of a block sorted by relative gain (desc; d c(v)
    for d >= 0, d / c(v) otherwise), then id; the shortest prefix covering the overload is selected;
    per target the selected nodes are admitted in ascending id while the target stays within its cap
    (round-start weights); then applied."""
    A = dense_adj(g)
    c = node_w(g)
    nb = len(wt)
    part, wt = part.copy(), wt.copy()
    rounds = 0
    contended = fallback = 0
    moved_prev = True
    while (wt > cap).any() and moved_prev:
        over = wt > cap
        free = [(int(cap[b] - wt[b]), -b) for b in range(nb) if not over[b]]
        tstar = -max(free)[1] if free else None
        conn = A @ np.eye(nb, dtype=np.int64)[part]
        cands = {}
        for v in range(g.n):
            b = int(part[v])
            if not over[b]:
                continue
            ts = [t for t in range(nb) if not over[t] and conn[v, t] > 0 and wt[t] + c[v] <= cap[t]]
            ts.sort(key=lambda t: (-int(conn[v, t]), oracle.hash_(seed, oracle.T_BAL, level, rounds, t), t))
            if ts:
                t = ts[0]
            elif tstar is not None and wt[tstar] + c[v] <= cap[tstar]:
                t = tstar
                fallback += 1
            else:
                continue
            d = int(conn[v, t] - conn[v, b])
            rg = fractions.Fraction(d * int(c[v])) if d >= 0 else fractions.Fraction(d, int(c[v]))
            cands.setdefault(b, []).append((-rg, v, t))
        sel = []
        for b, lst in cands.items():
            lst.sort()
            got = 0
            for _, v, t in lst:
                if got >= wt[b] - cap[b]:
                    break
                sel.append((t, v, b))
                got += int(c[v])
        sel.sort()
        room = {}
        nmoved = 0
        new_part, new_wt = part.copy(), wt.copy()
        for t, v, b in sel:
            room[t] = room.get(t, 0) + int(c[v])
            if wt[t] + room[t] <= cap[t]:
                new_part[v] = t
                new_wt[t] += c[v]
                new_wt[b] -= c[v]
                nmoved += 1
            else:
                contended += 1
        part, wt = new_part, new_wt
        rounds += 1
        moved_prev = nmoved > 0
    return part, wt, rounds, contended, fallback


@pytest.mark.parametrize("case", range(10))
def test_balance_rounds_restated(case):
    """Two or three overloaded blocks whose nodes compete for a target with little room; isolated nodes
    and nodes adjacent only to overloaded blocks take the most-free fallback."""
    rng = np.random.default_rng(60 + case)
    n, nb = 70, 5
    g = gen.random_graph(n, 3.0, 60 + case, max_vw=3, max_ew=4, isolated_frac=0.15)
    c = node_w(g)
    part = rng.integers(2, nb, n).astype(np.int32)
    part[: n // 4] = 0
    part[n // 4: n // 2] = 1
    wt = np.bincount(part, weights=c, minlength=nb).astype(np.int64)
    cap = wt.copy()
    cap[0] -= int(rng.integers(3, 9))
    cap[1] -= int(rng.integers(3, 9))
    if case % 3 == 0:
        cap[2] -= 2                              # a third overloaded block
    cap[3] += int(rng.integers(1, 4))           # a target with little room, wanted by several blocks
    cap[4] += 10 + case                         # the most free block: the fallback
    if case % 3 != 0:
        cap[2] += int(rng.integers(0, 3))
    exp_part, exp_wt, exp_rounds, contended, fallback = _balance(g, case % 3, 900 + case, part, wt, cap)
    got_part, got_wt, got_rounds = oracle.balance(g, case % 3, 900 + case, part, wt, cap)
    assert np.array_equal(got_part, exp_part), case
    assert np.array_equal(got_wt, exp_wt), case
    assert got_rounds == exp_rounds, case


def test_balance_cases_exercise_contention_and_fallback():
    tot_cont = tot_fb = multi = 0
    for case in range(10):
        rng = np.random.default_rng(60 + case)
        n, nb = 70, 5
        g = gen.random_graph(n, 3.0, 60 + case, max_vw=3, max_ew=4, isolated_frac=0.15)
        c = node_w(g)
        part = rng.integers(2, nb, n).astype(np.int32)
        part[: n // 4] = 0
        part[n // 4: n // 2] = 1
        wt = np.bincount(part, weights=c, minlength=nb).astype(np.int64)
        cap = wt.copy()
        cap[0] -= int(rng.integers(3, 9))
        cap[1] -= int(rng.integers(3, 9))
        if case % 3 == 0:
            cap[2] -= 2
        cap[3] += int(rng.integers(1, 4))
        cap[4] += 10 + case
        if case % 3 != 0:
            cap[2] += int(rng.integers(0, 3))
        _, _, rounds, cont, fb = _balance(g, case % 3, 900 + case, part, wt, cap)
        tot_cont += cont > 0
        tot_fb += fb > 0
        multi += rounds >= 2
    assert tot_cont >= 3 and tot_fb >= 3 and multi >= 1


def test_balance_fallback_tie_takes_smallest_index():
    """Isolated nodes of an overloaded block can only take the fallback; two non-overloaded blocks with
    equal free room tie, and the smaller index is the fallback."""
    from tests.helpers import csr_from_dense
    n = 12
    A = np.zeros((n, n), np.int64)
    for a, b in [(6, 7), (7, 8), (8, 9), (9, 10), (10, 11)]:
        A[a, b] = A[b, a] = 1
    g = csr_from_dense(A)
    part = np.array([0] * 6 + [1] * 3 + [2] * 3, np.int32)   # nodes 0..5 isolated in block 0
    wt = np.bincount(part, minlength=4).astype(np.int64)
    for room in (2, 3, 5):
        cap = np.array([3, 3 + room, 3 + room, room], np.int64)  # blocks 1 and 2 (and 3, empty) tie
        exp = _balance(g, 0, 5, part, wt, cap)
        got = oracle.balance(g, 0, 5, part, wt, cap)
        assert np.array_equal(got[0], exp[0]) and np.array_equal(got[1], exp[1]) and got[2] == exp[2]
        assert exp[4] > 0 and (exp[0][:6] == 1).sum() == min(3, room)
