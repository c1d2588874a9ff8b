"""GPU parity: every step of the HIP path through the C ABI against the CPU
oracle on the same seeded inputs.  All arithmetic is integer, so the bar is
bit-exact equality (labels, weights, favoured clusters, coarse CSR, block
tables, partitions, cuts)."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.helpers import csr_from_dense, node_w, two_cliques, with_hubs

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


def graphs_small():
    return [
        ("grid16", gen.grid(16, 16)),
        ("rand_w", gen.random_graph(600, 6.0, 11, max_vw=5, max_ew=7)),
        ("rand_iso", gen.random_graph(800, 3.0, 12, isolated_frac=0.2)),
        ("rgg3000", gen.rgg(3000, 8.0, 5)),
    ]


# ------------------------------------------------------------------ LP sub-round
@pytest.mark.parametrize("case", range(6))
def test_lp_subround(kmp, case):
    rng = np.random.default_rng(400 + case)
    name, g = graphs_small()[case % 4]
    n = g.n
    c = node_w(g)
    clustering = case < 3
    if clustering:
        nlab, tag = n, oracle.T_CL
        label = rng.integers(0, n, n).astype(np.int32)
        cap_scalar, capv = int(rng.integers(3, 20)), None
    else:
        nlab, tag = 6, oracle.T_REF
        label = rng.integers(0, nlab, n).astype(np.int32)
    wt = np.bincount(label, weights=c, minlength=nlab).astype(np.int64)
    if not clustering:
        capv = wt + rng.integers(0, 30, nlab)
        cap_scalar = 0
    active = (rng.random(n) < 0.7).astype(np.uint8) if case % 2 else None
    level, r, s = int(rng.integers(0, 4)), int(rng.integers(0, 5)), int(rng.integers(0, 4))
    seed = int(rng.integers(1, 2**40))
    say(f"[lp_subround] {name} case={case} clustering={clustering} level={level} r={r} s={s}")
    capo = capv if capv is not None else np.full(nlab, cap_scalar, np.int64)
    fav0 = np.full(n, 0xFFFFFFFF, np.uint32)
    exp_label, exp_wt, exp_fav, exp_moved, exp_nm = oracle.lp_subround(
        g, level, r, s, tag, seed, label, wt, capv=capo, active=active, fav=fav0)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    d_label, d_wt = t32(label), t64(wt)
    d_fav = t32(fav0.view(np.int32))
    d_moved = torch.zeros(n, dtype=torch.uint8, device="cuda")
    d_act = None if active is None else torch.from_numpy(active).cuda()
    d_cap = None if capv is None else t64(capv)
    nm = kmp.kmp_lp_subround(xadj, adjncy, vwgt, adjwgt, level, r, s, tag, seed, d_label, d_wt, d_cap, cap_scalar,
                             d_act, d_fav, d_moved)
    assert nm == exp_nm
    assert np.array_equal(d_label.cpu().numpy(), exp_label)
    assert np.array_equal(d_wt.cpu().numpy(), exp_wt)
    assert np.array_equal(d_moved.cpu().numpy(), exp_moved)
    assert np.array_equal(d_fav.cpu().numpy().view(np.uint32), exp_fav)


# ------------------------------------------------------------------ LP clustering
@pytest.mark.parametrize("gi", range(4))
def test_lp_cluster(kmp, gi):
    name, g = graphs_small()[gi]
    U, level, seed = 17, 1, 77
    say(f"[lp_cluster] {name} n={g.n} m={g.m}")
    exp_label, exp_cw, exp_fav, exp_moves, exp_rounds = oracle.lp_cluster(g, level, U, seed)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rounds, label, cw, fav, moves = kmp.kmp_lp_cluster(xadj, adjncy, vwgt, adjwgt, level, U, seed)
    assert rounds == exp_rounds
    assert moves == list(exp_moves)
    assert np.array_equal(label.cpu().numpy(), exp_label)
    assert np.array_equal(cw.cpu().numpy(), exp_cw)
    assert np.array_equal(fav.cpu().numpy().view(np.uint32), exp_fav)


def test_two_hop(kmp):
    for name, g in graphs_small():
        U, level, seed = 9, 0, 5
        label, cw, fav, _, _ = oracle.lp_cluster(g, level, U, seed)
        say(f"[two_hop] {name}")
        exp_label, exp_cw, exp_merged = oracle.two_hop(g, U, label, cw, fav)
        xadj, adjncy, vwgt, adjwgt = dev(g)
        d_label, d_cw, d_fav = t32(label), t64(cw), t32(fav.view(np.int32))
        merged = kmp.kmp_two_hop(xadj, adjncy, vwgt, adjwgt, U, d_label, d_cw, d_fav)
        assert merged == exp_merged
        assert np.array_equal(d_label.cpu().numpy(), exp_label)
        assert np.array_equal(d_cw.cpu().numpy(), exp_cw)


def _check_contract(kmp, g, label, name):
    say(f"[contract] {name} n={g.n} m={g.m}")
    exp_map, exp_cg = oracle.contract(g, label)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, mp, cx, ca, cv, cw = kmp.kmp_contract(xadj, adjncy, vwgt, adjwgt, t32(label))
    assert rc == 0
    assert np.array_equal(mp.cpu().numpy(), exp_map)
    assert np.array_equal(cx.cpu().numpy(), exp_cg.xadj)
    assert np.array_equal(ca.cpu().numpy(), exp_cg.adjncy)
    assert np.array_equal(cv.cpu().numpy(), exp_cg.vwgt)
    assert np.array_equal(cw.cpu().numpy(), exp_cg.adjwgt)


def test_contract_small(kmp):
    for name, g in graphs_small():
        label, cw, fav, _, _ = oracle.lp_cluster(g, 0, 13, 3)
        _check_contract(kmp, g, label, name)


def test_contract_heavy_rows(kmp):
    # clusters whose members carry > 4096 entries take the sort-reduce path;
    # random labels into few clusters make every row heavy
    rng = np.random.default_rng(3)
    g = gen.rgg(40000, 8.0, 9)
    _check_contract(kmp, g, rng.integers(0, 60, g.n).astype(np.int32), "rgg40000/60 clusters")
    _check_contract(kmp, g, rng.integers(0, 4000, g.n).astype(np.int32), "rgg40000/4000 clusters")
    gw = gen.random_graph(30000, 10.0, 4, max_vw=3, max_ew=9)
    _check_contract(kmp, gw, rng.integers(0, 25, gw.n).astype(np.int32), "weighted/25 clusters")


def hub_graphs():
    # degrees above 4096 take the one-workgroup-per-node tier with a global hash
    return [("rgg20000+hubs", with_hubs(gen.rgg(20000, 8.0, 5), [4097, 6000, 15000], seed=2)),
            ("rmat16", gen.rmat(16, 8 << 16, seed=3))]


@pytest.mark.parametrize("gi", range(2))
def test_hub_rating(kmp, gi):
    name, g = hub_graphs()[gi]
    assert int(np.diff(g.xadj).max()) > 4096
    for U, level, seed in ((6, 0, 9), (40, 2, 4)):
        say(f"[lp_cluster hubs] {name} maxdeg={int(np.diff(g.xadj).max())} U={U}")
        exp_label, exp_cw, exp_fav, exp_moves, exp_rounds = oracle.lp_cluster(g, level, U, seed)
        xadj, adjncy, vwgt, adjwgt = dev(g)
        rounds, label, cw, fav, moves = kmp.kmp_lp_cluster(xadj, adjncy, vwgt, adjwgt, level, U, seed)
        assert rounds == exp_rounds and moves == list(exp_moves)
        assert np.array_equal(label.cpu().numpy(), exp_label)
        assert np.array_equal(fav.cpu().numpy().view(np.uint32), exp_fav)
        _check_contract(kmp, g, exp_label, name)


@pytest.mark.parametrize("gi", range(2))
def test_hub_rating_small_lds_tables(kmp, gi):
    """Hub label partitions summed in 64-slot LDS tables: partitions of 64 or more entries try the LDS table
    and, with more distinct labels than slots, fall back to a global table of their own; the result is the
    oracle's either way."""
    name, g = hub_graphs()[gi]
    xadj, adjncy, vwgt, adjwgt = dev(g)
    try:
        t = kmp.kmp_get_tuning()
        assert kmp.kmp_set_tuning(dict(t, hub_lds_slots=64)) == kmp.KMP_OK
        for U, level, seed in ((6, 0, 9), (40, 2, 4)):
            say(f"[lp_cluster hubs, 64-slot LDS tables] {name} U={U}")
            exp_label, exp_cw, exp_fav, exp_moves, exp_rounds = oracle.lp_cluster(g, level, U, seed)
            rounds, label, cw, fav, moves = kmp.kmp_lp_cluster(xadj, adjncy, vwgt, adjwgt, level, U, seed)
            assert rounds == exp_rounds and moves == list(exp_moves)
            assert np.array_equal(label.cpu().numpy(), exp_label)
            assert np.array_equal(fav.cpu().numpy().view(np.uint32), exp_fav)
    finally:
        kmp.kmp_set_tuning(None)


# ------------------------------------------------------------------ bipartition, balance, refine
@pytest.mark.parametrize("k", [2, 5, 16])
def test_bipartition_round(kmp, k):
    g = gen.rgg(4000, 8.0, 21)
    lk = oracle.lk(g.n, k, 0.03)
    part = np.zeros(g.n, np.int32)
    first, fcount = [0], [k]
    d_part = t32(part)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    for rnd in range(4):
        if max(fcount) < 2:
            break
        say(f"[bipartition_round] k={k} round={rnd} blocks={len(first)}")
        part, ef, efc = oracle.bipartition_round(g, 0, part, first, fcount, lk, 3)
        rc, first, fcount = kmp.kmp_bipartition_round(xadj, adjncy, vwgt, adjwgt, 0, d_part, first, fcount, lk, 3)
        assert rc == 0
        assert first == list(ef) and fcount == list(efc)
        assert np.array_equal(d_part.cpu().numpy(), part)


def _heavy_nodes(n, seed):
    # 12% of the nodes weigh 50: near the end of a growth such frontier nodes no longer fit under the cap
    g = gen.random_graph(n, 4.0, seed)
    g.vwgt = np.where(np.random.default_rng(seed + 1).random(n) < 0.12, 50, 1).astype(np.int32)
    return g


def test_bipartition_weighted_and_degenerate(kmp):
    cases = [
        ("weighted", gen.random_graph(900, 5.0, 31, max_vw=20, max_ew=5), 7),
        ("heavy", _heavy_nodes(300, 33), 4),
        ("heavy-lds-and-global", _heavy_nodes(3000, 35), 6),
        # many internal entries per block: keys in LDS, entries in global memory (then LDS as blocks shrink)
        ("dense-hybrid", gen.random_graph(1200, 48.0, 38, max_ew=3), 5),
        ("cliques", csr_from_dense(two_cliques(40)), 2),
        ("tiny", gen.grid(1, 3), 8),
        ("isolated", gen.random_graph(500, 1.0, 32, isolated_frac=0.6), 4),
    ]
    for name, g, k in cases:
        lk = oracle.lk(int(node_w(g).sum()), k, 0.03)
        part = np.zeros(g.n, np.int32)
        first, fcount = [0], [k]
        d_part = t32(part)
        xadj, adjncy, vwgt, adjwgt = dev(g)
        while max(fcount) >= 2:
            say(f"[bipartition] {name} blocks={len(first)}")
            part, ef, efc = oracle.bipartition_round(g, 2, part, first, fcount, lk, 8)
            rc, first, fcount = kmp.kmp_bipartition_round(xadj, adjncy, vwgt, adjwgt, 2, d_part, first, fcount,
                                                          lk, 8)
            assert rc == 0 and first == list(ef) and fcount == list(efc)
            assert np.array_equal(d_part.cpu().numpy(), part)


@pytest.mark.parametrize("case", range(4))
def test_balance(kmp, case):
    rng = np.random.default_rng(600 + case)
    n, nb = 3000, 6
    g = gen.random_graph(n, 5.0, 600 + case, max_vw=1 if case < 2 else 6, max_ew=4)
    c = node_w(g)
    part = rng.integers(0, nb, n).astype(np.int32)
    part[: n // 3] = case % nb
    wt = np.bincount(part, weights=c, minlength=nb).astype(np.int64)
    cap = np.full(nb, int(c.sum()) // nb + 3, np.int64)
    say(f"[balance] case={case} overload={int((wt - cap).clip(0).sum())}")
    exp_part, exp_wt, exp_rounds = oracle.balance(g, 1, 44, part, wt, cap)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    d_part, d_wt = t32(part), t64(wt)
    rounds = kmp.kmp_balance(xadj, adjncy, vwgt, adjwgt, 1, 44, d_part, d_wt, t64(cap))
    assert rounds == exp_rounds
    assert np.array_equal(d_part.cpu().numpy(), exp_part)
    assert np.array_equal(d_wt.cpu().numpy(), exp_wt)


@pytest.mark.parametrize("gi", range(4))
def test_lp_refine(kmp, gi):
    name, g = graphs_small()[gi]
    rng = np.random.default_rng(700 + gi)
    nb = 5
    part = rng.integers(0, nb, g.n).astype(np.int32)
    c = node_w(g)
    wt = np.bincount(part, weights=c, minlength=nb).astype(np.int64)
    cap = wt + 10
    say(f"[lp_refine] {name}")
    exp_part, exp_wt, _, exp_moves, exp_rounds = oracle.lp_generic(g, 2, oracle.T_REF, 6, part, wt, capv=cap)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    d_part, d_wt = t32(part), t64(wt)
    rounds, moves = kmp.kmp_lp_refine(xadj, adjncy, vwgt, adjwgt, 2, 6, d_part, d_wt, t64(cap))
    assert rounds == exp_rounds and moves == list(exp_moves)
    assert np.array_equal(d_part.cpu().numpy(), exp_part)
    assert np.array_equal(d_wt.cpu().numpy(), exp_wt)


# ------------------------------------------------------------------ whole pipeline
def _e2e(kmp, g, k, eps, seed, name):
    say(f"[partition] {name} n={g.n} m={g.m} k={k} eps={eps} seed={seed}")
    ref = oracle.partition(g, k, eps, seed)
    rc, part, stats = kmp.partition(g, k, eps, seed)
    assert rc == ref.status
    assert np.array_equal(part, ref.part)
    assert stats["cut"] == ref.stats["cut"]
    assert stats["levels"] == ref.stats["levels"]
    assert stats["level_n"] == ref.stats["level_n"]
    assert stats["max_block_weight"] == ref.stats["max_block_weight"]
    return stats


@pytest.mark.parametrize("name,k,eps,seed", [
    ("grid128", 8, 0.03, 1), ("grid64", 3, 0.0, 2), ("rgg20000", 12, 0.03, 4), ("rgg20000", 64, 0.03, 1),
    ("rand_w", 7, 0.05, 9), ("rand_iso", 16, 0.03, 3), ("cliques", 2, 0.03, 1), ("grid16", 1, 0.03, 1),
    ("tiny", 8, 0.03, 1),
])
def test_partition_small(kmp, name, k, eps, seed):
    g = {
        "grid128": lambda: gen.grid(128, 128), "grid64": lambda: gen.grid(64, 64),
        "rgg20000": lambda: gen.rgg(20000, 8.0, 2),
        "rand_w": lambda: gen.random_graph(5000, 5.0, 7, max_vw=4, max_ew=6),
        "rand_iso": lambda: gen.random_graph(8000, 3.0, 8, isolated_frac=0.3),
        "cliques": lambda: csr_from_dense(two_cliques(200)), "grid16": lambda: gen.grid(16, 16),
        "tiny": lambda: gen.grid(2, 3),
    }[name]()
    _e2e(kmp, g, k, eps, seed, name)


@pytest.mark.parametrize("name,k", [("rgg20000", 16), ("rand_w", 7)])
def test_plain_loads_same_partition(kmp, name, k):
    """The lane rating kernel's plain-load path (graphs of 2^29 or more entries) gives the
    buffer-load path's partition, which is the oracle's."""
    g = {"rgg20000": lambda: gen.rgg(20000, 8.0, 2),
         "rand_w": lambda: gen.random_graph(5000, 5.0, 7, max_vw=4, max_ew=6)}[name]()
    say(f"[plain_loads] {name} k={k}")
    ref = oracle.partition(g, k, 0.03, 5)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    for plain in (False, True):
        rc, part, stats = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 5, plain_loads=plain)
        assert rc == ref.status
        assert np.array_equal(part.cpu().numpy(), ref.part)
        assert stats["cut"] == ref.stats["cut"]


def test_partition_validation_errors(kmp):
    g = gen.grid(8, 8)
    bad = gen.Graph(g.xadj.copy(), g.adjncy.copy())
    bad.adjncy[3] = 40   # breaks symmetry
    xadj, adjncy, _, _ = dev(bad)
    rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, None, None, 4, 0.03, 1, validate=True)
    assert rc == kmp.KMP_EGRAPH
    xadj, adjncy, _, _ = dev(g)
    rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, None, None, 4, 0.03, 1, validate=True)
    assert rc == kmp.KMP_OK
    big = torch.full((g.n,), 2**28, dtype=torch.int32, device="cuda")
    rc, _, _ = kmp.kmp_partition_ex(xadj, adjncy, big, None, 4, 0.03, 1)
    assert rc == kmp.KMP_EOVERFLOW


def test_partition_rgg_full(kmp):
    """RGG 2^20, k = 64: the benchmark workload, end to end."""
    g = gen.workload("rgg20")
    stats = _e2e(kmp, g, 64, 0.03, 1, "rgg20 (n=2^20)")
    say(f"  cut={stats['cut']} ms={stats['ms_total']:.1f}")


@pytest.mark.parametrize("gi,k", [(0, 8), (0, 64), (1, 16)])
def test_partition_hubs(kmp, gi, k):
    name, g = hub_graphs()[gi]
    _e2e(kmp, g, k, 0.03, 5, name)


@pytest.mark.parametrize("name,k,seed", [("grid128", 8, 1), ("rgg20000", 64, 1), ("rand_w", 7, 9), ("hubs", 8, 5)])
def test_partition_forced_exact_path(kmp, name, k, seed):
    """Every LP sub-round with a contended proposal stops on the device and is finished on the
    host-synchronised exact path (while the next round is already queued); the output must not
    change."""
    g = {"grid128": lambda: gen.grid(128, 128), "rgg20000": lambda: gen.rgg(20000, 8.0, 2),
         "rand_w": lambda: gen.random_graph(5000, 5.0, 7, max_vw=4, max_ew=6),
         "hubs": lambda: hub_graphs()[0][1]}[name]()
    say(f"[partition, exact path forced] {name} n={g.n} k={k} seed={seed}")
    ref = oracle.partition(g, k, 0.03, seed)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, part, stats = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, seed, force_exact=True)
    say(f"  exact sub-rounds: {stats['lp_exact_subrounds']}")
    assert rc == ref.status
    assert np.array_equal(part.cpu().numpy(), ref.part)
    assert stats["cut"] == ref.stats["cut"] and stats["level_n"] == ref.stats["level_n"]
    assert stats["lp_cluster_moves"] == ref.stats["lp_cluster_moves"]
    assert stats["lp_refine_moves"] == ref.stats["lp_refine_moves"]
    assert stats["lp_exact_subrounds"] > 0
    _, _, plain = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, seed)
    assert plain["lp_exact_subrounds"] < stats["lp_exact_subrounds"]


@pytest.mark.parametrize("name,k,seed,small", [("grid128", 8, 1, -1), ("rgg20000", 64, 1, -1),
                                               ("rgg20000", 12, 4, 1 << 22), ("rand_w", 7, 9, 1 << 22),
                                               ("hubs", 8, 5, 1 << 22), ("rand_iso", 16, 3, 1 << 22)])
def test_partition_lp_paths(kmp, name, k, seed, small):
    """LP calls on every level through the multi-launch path (small = -1), or on every level without
    a node of degree > 64 through the one-workgroup kernel (small = 2^22): the output is the oracle's."""
    g = {"grid128": lambda: gen.grid(128, 128), "rgg20000": lambda: gen.rgg(20000, 8.0, 2),
         "rand_w": lambda: gen.random_graph(5000, 5.0, 7, max_vw=4, max_ew=6),
         "rand_iso": lambda: gen.random_graph(8000, 3.0, 8, isolated_frac=0.3),
         "hubs": lambda: hub_graphs()[0][1]}[name]()
    say(f"[partition, small_level_n={small}] {name} n={g.n} k={k} seed={seed}")
    ref = oracle.partition(g, k, 0.03, seed)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    rc, part, stats = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, seed, small_level_n=small)
    assert rc == ref.status
    assert np.array_equal(part.cpu().numpy(), ref.part)
    assert stats["cut"] == ref.stats["cut"] and stats["level_n"] == ref.stats["level_n"]
    assert stats["lp_cluster_moves"] == ref.stats["lp_cluster_moves"]
    assert stats["lp_refine_moves"] == ref.stats["lp_refine_moves"]


@pytest.mark.parametrize("name,k", [("hubs", 8), ("rgg20000", 64)])
def test_partition_under_other_tunings(kmp, name, k):
    """Halved rating-tier cut-offs (more nodes in the wider tiers) and the one-workgroup LP off or on for
    every level: the output is the oracle's."""
    g = {"rgg20000": lambda: gen.rgg(20000, 8.0, 2), "hubs": lambda: hub_graphs()[0][1]}[name]()
    ref = oracle.partition(g, k, 0.03, 5)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    try:
        for small in (-1, 1 << 20):
            t = dict(small_level_n=small, tier0_deg=8, tier1_deg=32, tier2_deg=256, tier3_deg=2048,
                     hub_lds_slots=64 if small < 0 else 8192)
            assert kmp.kmp_set_tuning(t) == kmp.KMP_OK
            say(f"[partition, tuning {t}] {name} n={g.n} k={k}")
            rc, part, stats = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, 0.03, 5)
            assert rc == ref.status
            assert np.array_equal(part.cpu().numpy(), ref.part)
            assert stats["cut"] == ref.stats["cut"]
    finally:
        kmp.kmp_set_tuning(None)


def test_autotune_picks_a_setting_and_keeps_the_output(kmp):
    g = gen.rgg(20000, 8.0, 2)
    ref = oracle.partition(g, 16, 0.03, 3)
    xadj, adjncy, vwgt, adjwgt = dev(g)
    try:
        rc, chosen, report = kmp.kmp_autotune(xadj, adjncy, vwgt, adjwgt, 16, 0.03, 3, reps=2)
        say(f"[autotune] chosen {chosen} report {report}")
        assert rc == kmp.KMP_OK
        assert kmp.kmp_get_tuning() == chosen
        assert report["configs"] >= 10 and report["reps"] == 2
        assert 0 < report["ms_best"] <= report["ms_start"]
        rc, part, stats = kmp.kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, 16, 0.03, 3)
        assert rc == ref.status and np.array_equal(part.cpu().numpy(), ref.part)
    finally:
        kmp.kmp_set_tuning(None)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("case", sorted(f[:-5] for f in os.listdir(GOLDEN) if f.endswith(".json")))
def test_partition_golden(kmp, case):
    """Full-size workloads against stored oracle results (tests/golden/make_golden.py)."""
    exp = json.load(open(os.path.join(GOLDEN, case + ".json")))
    g = gen.workload(exp["workload"])
    gx = exp["graph"]
    assert (g.n, g.m) == (gx["n"], gx["m"])
    assert _sha(np.asarray(g.xadj, np.int32)) == gx["xadj_sha256"]
    assert _sha(np.asarray(g.adjncy, np.int32)) == gx["adjncy_sha256"]
    k = exp["k"]
    say(f"[golden] {case}: n={g.n} m={g.m} k={k}")
    opts = exp.get("options", {})
    rc, part, stats = kmp.partition(g, k, exp["eps"], exp["seed"], fm_passes=opts.get("fm_passes", 0),
                                    ip_pool=bool(opts.get("ip_pool", 0)),
                                    adaptive_eps=bool(opts.get("adaptive_eps", 0)),
                                    ip_multilevel=bool(opts.get("ip_multilevel", 0)))
    assert rc == exp["status"]
    bw = np.bincount(part, minlength=k).astype(np.int64)
    assert stats["cut"] == exp["stats"]["cut"]
    assert stats["levels"] == exp["stats"]["levels"]
    assert stats["level_n"] == exp["stats"]["level_n"]
    assert stats["level_m"] == exp["stats"]["level_m"]
    assert stats["max_block_weight"] == exp["stats"]["max_block_weight"]
    assert _sha(bw) == exp["block_weights_sha256"]
    assert _sha(np.asarray(part, np.int32)) == exp["part_sha256"]
    say(f"  cut={stats['cut']} ms={stats['ms_total']:.1f}")


# ------------------------------------------------------------------ batches
def _batch_jobs(specs):
    jobs = []
    for name, g, k, eps, seed in specs:
        xadj, adjncy, vwgt, adjwgt = dev(g)
        out = torch.full((max(g.n, 1),), -7, dtype=torch.int32, device="cuda")[:g.n]
        jobs.append(dict(name=name, g=g, xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, out=out, k=k,
                         epsilon=eps, seed=seed))
    return jobs


def _check_batch_against_oracle(kmp, jobs, skip=(), **kw):
    rc, res, _ = kmp.kmp_partition_batch(jobs, **kw)
    assert rc == kmp.KMP_OK
    for j, r in zip(jobs, res):
        if j["name"] in skip:
            continue
        ref = oracle.partition(j["g"], j["k"], j["epsilon"], j["seed"])
        say(f"  [batch job] {j['name']} n={j['g'].n} k={j['k']}: status {r['status']} cut {r['cut']}")
        assert r["status"] == ref.status, j["name"]
        assert np.array_equal(j["out"].cpu().numpy(), ref.part), j["name"]
        assert r["cut"] == ref.stats["cut"], j["name"]
        assert r["max_block_weight"] == ref.stats["max_block_weight"], j["name"]
        assert r["levels"] == ref.stats["levels"], j["name"]
        assert r["level_n"] == ref.stats["level_n"], j["name"]
    return res


def test_batch_mixed_jobs(kmp):
    """Jobs of different shapes, k, eps and seeds in one pass: each equals the oracle run alone."""
    specs = [
        ("grid64x40", gen.grid(64, 40), 8, 0.03, 3),
        ("rgg5000", gen.rgg(5000, 8.0, 7), 16, 0.03, 0),
        ("rand_w", gen.random_graph(3000, 5.0, 5, max_vw=4, max_ew=6), 5, 0.05, 9),
        ("rand_iso", gen.random_graph(4000, 3.0, 8, isolated_frac=0.3), 16, 0.03, 2),
        ("tiny", gen.grid(2, 3), 8, 0.03, 1),
        ("k1", gen.grid(16, 16), 1, 0.03, 4),
        ("grid128", gen.grid(128, 128), 8, 0.03, 1),
        ("rgg20000", gen.rgg(20000, 8.0, 2), 64, 0.03, 1),
        ("hubs", with_hubs(gen.rgg(20000, 8.0, 5), [4097, 6000, 15000], seed=2), 8, 0.03, 5),
        ("cliques", csr_from_dense(two_cliques(100)), 2, 0.03, 1),
        ("rgg700_eps0", gen.rgg(700, 8.0, 3), 4, 0.0, 6),
    ]
    say(f"[batch] {len(specs)} mixed jobs")
    _check_batch_against_oracle(kmp, _batch_jobs(specs))


def test_batch_forced_exact_path(kmp):
    """The batch pass with the exact admission path forced for every contended sub-round."""
    specs = [
        ("grid64x40", gen.grid(64, 40), 8, 0.03, 3),
        ("rgg5000", gen.rgg(5000, 8.0, 7), 16, 0.03, 0),
        ("rand_w", gen.random_graph(3000, 5.0, 5, max_vw=4, max_ew=6), 5, 0.05, 9),
        ("tiny", gen.grid(2, 3), 8, 0.03, 1),
    ]
    say(f"[batch, exact path forced] {len(specs)} jobs")
    _check_batch_against_oracle(kmp, _batch_jobs(specs), force_exact=True)


@pytest.mark.parametrize("small", [-1, 1 << 22])
def test_batch_lp_paths(kmp, small):
    """The batch pass with every LP call on the multi-launch path, or on the one-workgroup kernel
    wherever the union level qualifies."""
    specs = [
        ("grid64x40", gen.grid(64, 40), 8, 0.03, 3),
        ("rgg5000", gen.rgg(5000, 8.0, 7), 16, 0.03, 0),
        ("rand_w", gen.random_graph(3000, 5.0, 5, max_vw=4, max_ew=6), 5, 0.05, 9),
        ("rand_iso", gen.random_graph(4000, 3.0, 8, isolated_frac=0.3), 16, 0.03, 2),
        ("tiny", gen.grid(2, 3), 8, 0.03, 1),
    ]
    say(f"[batch, small_level_n={small}] {len(specs)} jobs")
    _check_batch_against_oracle(kmp, _batch_jobs(specs), small_level_n=small)


def test_batch_errors_and_empty_jobs(kmp):
    """Bad jobs get their own status and do not disturb the others."""
    good = gen.grid(20, 20)
    specs = [("good0", good, 4, 0.03, 1), ("empty", gen.Graph(np.zeros(1, np.int32), np.zeros(0, np.int32)), 4,
                                                                0.03, 1),
             ("good1", gen.rgg(3000, 8.0, 1), 8, 0.03, 2)]
    jobs = _batch_jobs(specs)
    bad = _batch_jobs([("bad_m", good, 4, 0.03, 1)])[0]
    bad["adjncy"] = torch.cat([bad["adjncy"], bad["adjncy"][:1]])  # m != xadj[n]
    bad_k = _batch_jobs([("bad_k", good, 0, 0.03, 1)])[0]
    heavy = gen.grid(8, 8)
    over = _batch_jobs([("overflow", gen.Graph(heavy.xadj, heavy.adjncy, np.full(64, 2**28, np.int32)), 4, 0.03,
                         1)])[0]
    jobs = [jobs[0], bad, jobs[1], bad_k, over, jobs[2]]
    rc, res, _ = kmp.kmp_partition_batch(jobs)
    assert rc == kmp.KMP_OK
    assert [r["status"] for r in res] == [0, kmp.KMP_EINVAL, 0, kmp.KMP_EINVAL, kmp.KMP_EOVERFLOW, 0]
    for j in (jobs[0], jobs[5]):
        ref = oracle.partition(j["g"], j["k"], j["epsilon"], j["seed"])
        assert np.array_equal(j["out"].cpu().numpy(), ref.part)


def test_batch_workload_sample(kmp):
    """32 graphs of the batched recipe (grids and RGGs, n log-uniform in [2^10, 2^13]), k = 16."""
    sizes = gen.batch_sizes(32, lo=10, span=3)
    specs = [(f"b{i}", gen.batch_graph(i, n), 16, 0.03, i) for i, n in enumerate(sizes)]
    say(f"[batch] recipe sample, sum n = {sum(sizes)}")
    _check_batch_against_oracle(kmp, _batch_jobs(specs))


def test_batch_equals_single_calls(kmp):
    """The same job alone (kmp_partition_ex) and inside a batch gives the same partition."""
    specs = [(f"r{i}", gen.rgg(2000 + 700 * i, 8.0, 40 + i), 8 + i, 0.03, 100 + i) for i in range(6)]
    jobs = _batch_jobs(specs)
    rc, res, _ = kmp.kmp_partition_batch(jobs)
    assert rc == 0
    for j, r in zip(jobs, res):
        rc1, out1, st1 = kmp.kmp_partition_ex(j["xadj"], j["adjncy"], j["vwgt"], j["adjwgt"], j["k"], j["epsilon"],
                                              j["seed"])
        assert rc1 == r["status"]
        assert torch.equal(out1, j["out"])
        assert st1["cut"] == r["cut"]


def test_batch_beyond_2_28_entries(kmp):
    """A batch whose union holds more than 2^28 directed entries (more threads than a 2^20-block grid
    covers): every job equals its single kmp_partition_ex call, which the golden tests pin to the oracle."""
    rm = gen.rmat(21, 8 << 21, seed=21)
    rg = gen.rgg(1 << 20, 8.0, seed=1)
    specs = [(f"rmat21_{i}", rm, (2, 64, 512, 4096)[i % 4], 0.03, 50 + i) for i in range(9)]
    specs += [("rgg20_a", rg, 64, 0.03, 1), ("rgg20_b", rg, 8, 0.03, 2)]
    total = sum(g.m for _, g, _, _, _ in specs)
    assert total > (1 << 28)
    say(f"[batch] {len(specs)} jobs, sum m = {total}")
    jobs = _batch_jobs(specs)
    rc, res, _ = kmp.kmp_partition_batch(jobs)
    assert rc == kmp.KMP_OK
    for j, r in zip(jobs, res):
        rc1, out1, st1 = kmp.kmp_partition_ex(j["xadj"], j["adjncy"], j["vwgt"], j["adjwgt"], j["k"], j["epsilon"],
                                              j["seed"])
        assert rc1 == r["status"], j["name"]
        assert st1["cut"] == r["cut"], j["name"]
        assert torch.equal(out1, j["out"]), j["name"]
