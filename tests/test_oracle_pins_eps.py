"""Pins of the oracle's adaptive imbalance (O8d): Sec. 2 ("Maintaining the
Balance Constraint") and Alg. 2 give eps' = ((1 + eps) c(V)/k * k'/c(V'))^(1/ceil(log2 k')) - 1
for a subgraph V' that is to end as k' blocks, and Sec. 5.2 bounds a side by
(1 + eps') ceil(c(V')/2).  The oracle evaluates the root in 2^32 fixed point
(the largest q whose stepwise-floored r-th power stays within the floored
scaled radicand); these tests check it against exact powers, against the
real root within the error the flooring allows, and the caps against the
real-valued bound."""
import fractions
import math

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.helpers import node_w

ONE = 1 << 32


def test_root_exact_powers():
    assert oracle.eps_root(ONE, 1) == ONE
    for r in range(1, 8):
        assert oracle.eps_root(ONE, r) == ONE                 # eps' = 0 when the radicand is 1
        assert oracle.eps_root(ONE << r, r) == 2 * ONE        # 2^r -> 2
        assert oracle.eps_root(ONE * 3 ** r, r) == 3 * ONE    # 3^r -> 3
    for x in (0, 1, 12345, ONE - 1, ONE + 1, 5 * ONE + 17, (1 << 63) + 5):
        assert oracle.eps_root(x, 1) == x                     # r = 1: the radicand itself


def _real_root(x, r):
    """x / 2^32 to the power 1/r, as a float with enough headroom for the bound below."""
    return math.exp(math.log(x / ONE) / r) if x > 0 else 0.0


@pytest.mark.parametrize("r", [1, 2, 3, 5, 8, 15])
def test_root_within_flooring_error_and_maximal(r):
    rng = np.random.default_rng(r)
    for _ in range(40):
        x = int(rng.integers(ONE // 4, 40 * ONE))
        q = oracle.eps_root(x, r)
        real = _real_root(x, r) * ONE
        # the radicand is floored once and each of the r power steps floors once, so the fixed-point
        # root is within r + 2 units (of 2^-32, scaled by the root) of the real one
        tol = (r + 2) * max(1.0, real / ONE) + 1
        assert abs(q - real) <= tol
    # the exact definition: P(q) <= x < P(q + 1) with P the stepwise-floored power
    def P(q):
        p = ONE
        for _ in range(r):
            p = (p * q) >> 32
        return p
    for x in (ONE, 3 * ONE + 7, 11 * ONE // 3, 2 ** 40):
        q = oracle.eps_root(x, r)
        assert P(q) <= x < P(q + 1)


def test_caps_closed_form():
    # eps = 0, k = 4, a block of weight 256 out of 1024 that must end as 4 blocks:
    # (1 + eps')^2 = (1024 / 4) * (4 / 256) = 4, so 1 + eps' = 2 and each side's bound is 2 * ceil(256 * 2 / 4)
    assert oracle.adaptive_caps(1024, 4, 0.0, 256, 4) == (256, 256)
    # f = 3 (r = 2), sides 1 and 2 of 3: X = (900/3) * (3 / 100) = 9 -> 1 + eps' = 3, T = (34, 67)
    assert oracle.adaptive_caps(900, 3, 0.0, 100, 3) == (3 * 34, 3 * 67)
    # a block exactly at its share with eps = 0: eps' = 0, the caps are the ceilings of the shares
    assert oracle.adaptive_caps(1000, 8, 0.0, 500, 4) == (250, 250)
    # empty block; an unbounded case (tiny block, huge radicand)
    assert oracle.adaptive_caps(1000, 8, 0.03, 0, 4) == (0, 0)
    c0, c1 = oracle.adaptive_caps(2**31 - 1, 2, 2.0, 1, 2)  # (1 + eps')^1 = 3 (2^31 - 1) >= 2^32
    assert c0 == c1 == 1 << 62


@pytest.mark.parametrize("seed", range(6))
def test_caps_follow_the_real_bound(seed):
    """cap_j = floor((1 + eps') ceil(c(B) f_j / f)) up to the fixed-point error: never above the real bound
    and at most one unit plus the root's error below it."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(60):
        k = int(rng.integers(2, 5000))
        cV = int(rng.integers(k, 2**31 - 1))
        f = int(rng.integers(2, k + 1))
        cB = int(rng.integers(1, cV + 1))
        eps = float(rng.choice([0.0, 0.01, 0.03, 0.1, 1.0]))
        e = oracle.eps_ppm(eps)
        r = (f - 1).bit_length()
        X = fractions.Fraction((10**6 + e) * cV * f, 10**6 * k * cB)
        if X >= 2**32:
            continue
        root = math.exp(math.log(float(X)) / r)
        f0, f1 = f // 2, f - f // 2
        caps = oracle.adaptive_caps(cV, k, eps, cB, f)
        for fj, cap in zip((f0, f1), caps):
            T = -(-cB * fj // f)
            real = root * T
            slack = T * (r + 3) * root / ONE + 1e-6 * real
            assert cap <= real + slack
            assert cap >= real - 1 - slack


def test_top_level_block_gets_eps_root():
    """The whole graph about to be split into k blocks: eps' = (1 + eps)^(1/ceil(log2 k)) - 1 (Sec. 2)."""
    for k, eps in ((4, 0.21), (8, 0.331), (2, 0.03), (64, 0.03)):
        cV = 1_000_000
        c0, c1 = oracle.adaptive_caps(cV, k, eps, cV, k)
        r = (k - 1).bit_length()
        one_eps = (1 + eps) ** (1 / r)
        assert abs(c0 - one_eps * (cV // 2)) <= 1 + cV * 1e-9
        assert abs(c1 - one_eps * (cV // 2)) <= 1 + cV * 1e-9


@pytest.mark.parametrize("name,k", [("grid", 8), ("rgg", 12), ("weighted", 7), ("rmat", 32)])
def test_partition_with_adaptive_caps(name, k):
    """Whole partitions with the adaptive caps: valid, every bipartition within its caps is checked by
    the restated round below, and unit-weight inputs end balanced."""
    g = {"grid": lambda: gen.grid(60, 60), "rgg": lambda: gen.rgg(6000, 8.0, 4),
         "weighted": lambda: gen.random_graph(3000, 5.0, 9, max_vw=6, max_ew=4),
         "rmat": lambda: gen.rmat(13, 8 << 13, seed=2)}[name]()
    ref = oracle.partition(g, k, 0.03, 1, adaptive_eps=True)
    base = oracle.partition(g, k, 0.03, 1)
    assert ref.status in (0, 1)
    assert set(np.unique(ref.part)) <= set(range(k))
    if g.vwgt is None:
        assert ref.status == 0 and ref.stats["max_block_weight"] <= oracle.lk(g.n, k, 0.03)
    # the option changes the caps of the bipartitions, so in general the partition
    assert ref.stats["cut"] > 0 and base.stats["cut"] > 0


def test_bipartition_round_uses_adaptive_caps():
    """One round restated: each block's GGG run with the caps of O8d gives the same sides."""
    g = gen.random_graph(400, 5.0, 21, max_vw=4, max_ew=3)
    c = node_w(g)
    cV, k, eps = int(c.sum()), 7, 0.03
    lk_ = oracle.lk(cV, k, eps)
    part = np.zeros(g.n, np.int32)
    got, first, f = oracle.bipartition_round(g, 1, part, [0], [k], lk_, 5, adaptive=(cV, k, eps))
    caps = oracle.adaptive_caps(cV, k, eps, cV, k)
    side, _ = oracle.ggg(g, 1, 0, k, lk_, 5, caps=caps)
    assert np.array_equal(got, side.astype(np.int32))
    assert list(first) == [0, 3] and list(f) == [3, 4]
    # with the default caps the sides may differ; the adaptive caps are tighter than f_j L_k here
    assert caps[0] <= 3 * lk_ and caps[1] <= 4 * lk_


def test_ggg_respects_given_caps():
    """GGG with the adaptive caps keeps both sides within them whenever a run is feasible, and on inputs with
    heavy nodes the caps change the chosen bipartition compared with the f_j L_k caps."""
    differ = 0
    for seed in range(12):
        g = gen.random_graph(120, 4.0, 300 + seed, max_vw=9, max_ew=3)
        c = node_w(g)
        cB, k, f, eps = int(c.sum()), 16, 4, 0.03
        # the graph is a block that must end as f of k blocks but weighs 20% more than its share
        cV = int(cB * k / f / 1.2)
        lk_ = oracle.lk(cV, k, eps)
        caps = oracle.adaptive_caps(cV, k, eps, cB, f)
        side, _ = oracle.ggg(g, 0, 0, f, lk_, 11 + seed, caps=caps)
        side_d, _ = oracle.ggg(g, 0, 0, f, lk_, 11 + seed)
        w0 = int(c[side == 0].sum())
        over = max(0, w0 - caps[0]) + max(0, cB - w0 - caps[1])
        over_default_caps = max(0, int(c[side_d == 0].sum()) - caps[0]) + \
            max(0, cB - int(c[side_d == 0].sum()) - caps[1])
        assert over <= over_default_caps   # the kept run minimises the overload against the given caps
        differ += not np.array_equal(side, side_d)
    assert differ >= 1
