"""CPU oracle for deep multilevel graph partitioning -- TEST INFRASTRUCTURE.

Plain single-threaded C (``kmp_oracle.c``) wrapped with ctypes.  Only the
tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg
may import this package; the HIP library never does.

Every function follows one step of the deterministic reading of the paper
(see the step list at the top of ``kmp_oracle.c``).  Graphs are
``paper_2105_02022_amd.gen.Graph`` objects (numpy int32 CSR); missing
weights mean unit weights.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kmp_oracle.c")
_LIB = os.path.join(_HERE, "libkmp_oracle.so")

C = 160
ROUNDS = 5
S = 4
R = 8
PPM = 1_000_000
NONE = 0xFFFFFFFF
T_SUB, T_CL, T_REF, T_BAL, T_GGG, T_BFS, T_RND = 1, 2, 3, 4, 5, 6, 7

OK, IMBALANCED, EINVAL, EGRAPH, EOVERFLOW, ENOMEM = 0, 1, -1, -2, -3, -4

TRACE_PHASES = {
    1: "cluster", 2: "twohop", 3: "map", 4: "coarse_xadj", 5: "coarse_adjncy", 6: "coarse_vwgt",
    7: "coarse_adjwgt", 8: "project", 9: "bipart", 10: "balance", 11: "refine", 12: "first", 13: "fcount",
}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (plain C, single-threaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Stats(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("level_n", ctypes.c_int32 * 65), ("level_m", ctypes.c_int64 * 65),
                ("bipartitions", ctypes.c_int32), ("balance_rounds", ctypes.c_int32),
                ("lp_cluster_moves", ctypes.c_int64), ("lp_refine_moves", ctypes.c_int64),
                ("max_block_weight", ctypes.c_int64), ("lk", ctypes.c_int64)]


TRACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int32), ctypes.c_int64)

_lib = None
P32 = ctypes.POINTER(ctypes.c_int32)
P64 = ctypes.POINTER(ctypes.c_int64)
PU32 = ctypes.POINTER(ctypes.c_uint32)
PU8 = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32, i64, u64, u32, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        sig = {
            "or_fmix32": (u32, [u32]),
            "or_hash": (u32, [u64, i32, PU32]),
            "or_eps_ppm": (i64, [dbl]),
            "or_lk": (i64, [i64, i32, i64]),
            "or_level_U": (i64, [i32, P32, i64, i64]),
            "or_validate": (ctypes.c_int, [i32, P32, P32, P32, P32]),
            "or_partition_traced": (ctypes.c_int, [i32, P32, P32, P32, P32, i32, dbl, u64, P32,
                                                   ctypes.POINTER(Stats), ctypes.c_int, TRACE_FN,
                                                   ctypes.c_void_p, i32, i32]),
            "or_step_lp_cluster": (i32, [i32, P32, P32, P32, P32, i32, i64, u64, P32, P64, PU32, P64]),
            "or_step_lp_generic": (i32, [i32, P32, P32, P32, P32, i32, u32, u64, P32, P64, i32, P64, i64,
                                         PU32, P64]),
            "or_step_lp_async": (i32, [i32, P32, P32, P32, P32, i32, u32, u64, P32, P64, i32, P64, i64,
                                       PU32, P64]),
            "or_step_two_hop": (i64, [i32, P32, P32, P32, P32, i64, P32, P64, PU32]),
            "or_step_contract": (ctypes.c_int, [i32, P32, P32, P32, P32, P32, P32, P32, P64, P32, P32, P32,
                                                P32]),
            "or_step_bipartition_round": (ctypes.c_int, [i32, P32, P32, P32, P32, i32, P32, P32, P32, P32,
                                                         i64, u64, i32, i32, i64, i32, i64]),
            "or_ggg": (ctypes.c_int, [i32, P32, P32, P32, P32, i32, i32, i32, i64, u64, PU8, P64, i32, i32]),
            "or_fm2_stall": (ctypes.c_int, [i32, P32, P32, P32, P32, PU8, i64, i64, i32, i32, P64]),
            "or_step_balance": (i32, [i32, P32, P32, P32, P32, i32, u64, P32, P64, i32, P64]),
            "or_step_balance_pq": (i32, [i32, P32, P32, P32, P32, i32, u64, P32, P64, i32, P64]),
            "or_step_cut": (i64, [i32, P32, P32, P32, P32]),
            "or_ggg_traced": (ctypes.c_int, [i32, P32, P32, P32, P32, i32, i32, i32, i64, u64, PU8, P64, P32,
                                             P32, P32, i32, i32, i64, i64]),
            "or_ml_bipartition": (ctypes.c_int, [i32, P32, P32, P32, P32, i32, i32, i32, i64, u64, PU8, i32, i32,
                                                 i64, i64, P32]),
            "or_eps_root": (u64, [u64, i32]),
            "or_adaptive_caps": (None, [i64, i32, i64, i64, i32, P64, P64]),
            "or_rg_cmp": (ctypes.c_int, [i64, i64, i64, i64]),
            "or_step_lp_subround": (i64, [i32, P32, P32, P32, P32, i32, i32, i32, u32, u64, P32, P64, i32, P64,
                                          i64, PU8, PU32, PU8]),
            "or_set_visit_order": (None, [ctypes.c_int]),
            "or_sub_class": (u32, [u64, i32, i32]),
            "or_count_labels": (i32, [i32, P32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a, typ=P32):
    if a is None:
        return None
    return a.ctypes.data_as(typ)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _weights(g):
    n, m = g.n, g.m
    vw = _i32(g.vwgt) if g.vwgt is not None else np.ones(n, np.int32)
    ew = _i32(g.adjwgt) if g.adjwgt is not None else np.ones(m, np.int32)
    return vw, ew


# ---------------------------------------------------------------- scalars

def fmix32(h: int) -> int:
    return int(_load().or_fmix32(h & 0xFFFFFFFF))


def hash_(seed: int, *args: int) -> int:
    a = np.array([x & 0xFFFFFFFF for x in args], dtype=np.uint32)
    return int(_load().or_hash(seed & (2**64 - 1), len(args), _p(a, PU32)))


def eps_ppm(eps: float) -> int:
    return int(_load().or_eps_ppm(eps))


def lk(cV: int, k: int, eps: float) -> int:
    return int(_load().or_lk(cV, k, eps_ppm(eps)))


def level_U(n_l: int, kc: int, cV: int, eps: float) -> Tuple[int, int]:
    """U_l and the updated k'_c for a level with n_l nodes."""
    kk = ctypes.c_int32(kc)
    u = _load().or_level_U(n_l, ctypes.byref(kk), cV, eps_ppm(eps))
    return int(u), int(kk.value)


def validate(g) -> int:
    return int(_load().or_validate(g.n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)),
                                   _p(None if g.vwgt is None else _i32(g.vwgt)),
                                   _p(None if g.adjwgt is None else _i32(g.adjwgt))))


# ---------------------------------------------------------------- driver

@dataclass
class Result:
    status: int
    part: np.ndarray
    stats: Dict
    trace: Dict[Tuple[str, int], np.ndarray] = field(default_factory=dict)


IP_POOL, IP_ADAPTIVE, BAL_PQ, LP_ASYNC, IP_ML = 1, 2, 4, 8, 16
IP_CCF, IP_MAXLEV = 18, 32


def _ipflags(pool, adaptive_eps, pq_balance=False, async_lp=False, ml=False):
    return (IP_POOL if pool else 0) | (IP_ADAPTIVE if adaptive_eps else 0) | (BAL_PQ if pq_balance else 0) | \
        (LP_ASYNC if async_lp else 0) | (IP_ML if ml else 0)


def partition(g, k: int, eps: float = 0.03, seed: int = 1, trace: bool = False,
              validate_input: bool = True, fm_passes: int = 0, pool: bool = False,
              adaptive_eps: bool = False, pq_balance: bool = False, async_lp: bool = False,
              ip_multilevel: bool = False) -> Result:
    """O10; async_lp: every LP call is the one-PE execution of the asynchronous LP (O3b); ip_multilevel:
    every bipartition is the multilevel one of O8e."""
    lib = _load()
    xadj, adjncy = _i32(g.xadj), _i32(g.adjncy)
    vw = None if g.vwgt is None else _i32(g.vwgt)
    ew = None if g.adjwgt is None else _i32(g.adjwgt)
    out = np.zeros(max(g.n, 1), np.int32)
    st = Stats()
    tr: Dict[Tuple[str, int], np.ndarray] = {}

    def _cb(user, phase, level, data, length):
        arr = np.ctypeslib.as_array(data, shape=(max(int(length), 1),))[:int(length)].copy() \
            if length > 0 else np.zeros(0, np.int32)
        tr[(TRACE_PHASES[int(phase)], int(level))] = arr

    cb = TRACE_FN(_cb) if trace else TRACE_FN()
    rc = lib.or_partition_traced(g.n, _p(xadj), _p(adjncy), _p(vw), _p(ew), k, eps, seed & (2**64 - 1),
                                 _p(out), ctypes.byref(st), int(validate_input), cb, None, int(fm_passes),
                                 _ipflags(pool, adaptive_eps, pq_balance, async_lp, ip_multilevel))
    L = st.levels
    stats = dict(cut=st.cut, levels=L, level_n=list(st.level_n[:L + 1]), level_m=list(st.level_m[:L + 1]),
                 bipartitions=st.bipartitions, balance_rounds=st.balance_rounds,
                 lp_cluster_moves=st.lp_cluster_moves, lp_refine_moves=st.lp_refine_moves,
                 max_block_weight=st.max_block_weight, lk=st.lk)
    return Result(int(rc), out[:g.n], stats, tr)


# ---------------------------------------------------------------- steps

def lp_cluster(g, level: int, U: int, seed: int):
    """O3 clustering from singletons; returns (label, cluster weights, fav, moves per round, rounds)."""
    vw, ew = _weights(g)
    n = g.n
    label = np.zeros(max(n, 1), np.int32)
    cw = np.zeros(max(n, 1), np.int64)
    fav = np.zeros(max(n, 1), np.uint32)
    moves = np.zeros(ROUNDS, np.int64)
    r = _load().or_step_lp_cluster(n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), level, U,
                                   seed, _p(label), _p(cw, P64), _p(fav, PU32), _p(moves, P64))
    return label[:n], cw[:n], fav[:n], moves, int(r)


def lp_generic(g, level: int, tag: int, seed: int, label, wt, capv=None, caps: int = 0, fav=None):
    """O3 from an arbitrary state; label/wt/fav are updated in place copies and returned."""
    vw, ew = _weights(g)
    label = _i32(label).copy()
    wt = np.ascontiguousarray(wt, dtype=np.int64).copy()
    favv = None if fav is None else np.ascontiguousarray(fav, dtype=np.uint32).copy()
    capv = None if capv is None else np.ascontiguousarray(capv, dtype=np.int64)
    moves = np.zeros(ROUNDS, np.int64)
    r = _load().or_step_lp_generic(g.n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), level, tag,
                                   seed, _p(label), _p(wt, P64), int(wt.shape[0]), _p(capv, P64), caps,
                                   _p(favv, PU32), _p(moves, P64))
    return label, wt, favv, moves, int(r)


def lp_async(g, level: int, tag: int, seed: int, label, wt, capv=None, caps: int = 0, fav=None):
    """O3b (asynchronous LP executed by one PE, visits by degree bucket) from an arbitrary state; returns
    (label, wt, fav, moves per round, rounds) like lp_generic."""
    vw, ew = _weights(g)
    label = _i32(label).copy()
    wt = np.ascontiguousarray(wt, dtype=np.int64).copy()
    favv = None if fav is None else np.ascontiguousarray(fav, dtype=np.uint32).copy()
    capv = None if capv is None else np.ascontiguousarray(capv, dtype=np.int64)
    moves = np.zeros(ROUNDS, np.int64)
    r = _load().or_step_lp_async(g.n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), level, tag,
                                 seed, _p(label), _p(wt, P64), int(wt.shape[0]), _p(capv, P64), caps,
                                 _p(favv, PU32), _p(moves, P64))
    return label, wt, favv, moves, int(r)


def two_hop(g, U: int, label, cw, fav):
    vw, ew = _weights(g)
    label = _i32(label).copy()
    cw = np.ascontiguousarray(cw, dtype=np.int64).copy()
    fav = np.ascontiguousarray(fav, dtype=np.uint32)
    merged = _load().or_step_two_hop(g.n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), U,
                                     _p(label), _p(cw, P64), _p(fav, PU32))
    return label, cw, int(merged)


def contract(g, label):
    from paper_2105_02022_amd.gen import Graph
    vw, ew = _weights(g)
    n, m = g.n, g.m
    mp = np.zeros(max(n, 1), np.int32)
    cn = ctypes.c_int32(0)
    cm = ctypes.c_int64(0)
    cx = np.zeros(n + 1, np.int32)
    ca = np.zeros(max(m, 1), np.int32)
    cv = np.zeros(max(n, 1), np.int32)
    cw = np.zeros(max(m, 1), np.int32)
    rc = _load().or_step_contract(n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), _p(_i32(label)),
                                  _p(mp), ctypes.byref(cn), ctypes.byref(cm), _p(cx), _p(ca), _p(cv), _p(cw))
    if rc != 0:
        raise RuntimeError(f"oracle contract failed: {rc}")
    nc, mc = cn.value, cm.value
    return mp[:n], Graph(cx[:nc + 1].copy(), ca[:mc].copy(), cv[:nc].copy(), cw[:mc].copy(), "coarse")


def bipartition_round(g, level: int, part, first, fcount, lk_: int, seed: int, fm_passes: int = 0,
                      pool: bool = False, adaptive: Optional[Tuple[int, int, float]] = None, ml: bool = False):
    """O7 round; `adaptive` = (c(V), k, eps) bounds each side by the adaptive imbalance (O8d)."""
    vw, ew = _weights(g)
    part = _i32(part).copy()
    nb = ctypes.c_int32(len(first))
    cap = 2 * len(first) + 1
    fa = np.zeros(cap, np.int32)
    fc = np.zeros(cap, np.int32)
    fa[:len(first)] = first
    fc[:len(first)] = fcount
    rc = _load().or_step_bipartition_round(g.n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), level,
                                           _p(part), ctypes.byref(nb), _p(fa), _p(fc), lk_, seed, int(fm_passes),
                                           _ipflags(pool, adaptive is not None, ml=ml),
                                           adaptive[0] if adaptive else 0, adaptive[1] if adaptive else 1,
                                           eps_ppm(adaptive[2]) if adaptive else 0)
    if rc != 0:
        raise RuntimeError(f"oracle bipartition failed: {rc}")
    q = nb.value
    return part, fa[:q].copy(), fc[:q].copy()


def ggg(sub, level: int, first: int, f: int, lk_: int, seed: int, with_order: bool = False, fm_passes: int = 0,
        pool: bool = False, caps: Optional[Tuple[int, int]] = None):
    """O8 (with O8b when fm_passes > 0, O8c when pool) on a subgraph given in local ids; returns (side, cut)
    or (side, cut, growth order of the kept run, index q = algorithm * R + j of the kept run)."""
    vw, ew = _weights(sub)
    side = np.zeros(max(sub.n, 1), np.uint8)
    cut = ctypes.c_int64(0)
    order = np.zeros(max(sub.n, 1), np.int32)
    norder = ctypes.c_int32(0)
    jbest = ctypes.c_int32(-1)
    rc = _load().or_ggg_traced(sub.n, _p(_i32(sub.xadj)), _p(_i32(sub.adjncy)), _p(ew), _p(vw), level, first, f,
                               lk_, seed, _p(side, PU8), ctypes.byref(cut), _p(order), ctypes.byref(norder),
                               ctypes.byref(jbest), int(fm_passes), int(pool), -1 if caps is None else caps[0],
                               -1 if caps is None else caps[1])
    if rc != 0:
        raise RuntimeError(f"oracle ggg failed: {rc}")
    if with_order:
        return side[:sub.n], int(cut.value), order[:norder.value].copy(), int(jbest.value)
    return side[:sub.n], int(cut.value)


def ml_bipartition(sub, level: int, first: int, f: int, lk_: int, seed: int, fm_passes: int = 0,
                   pool: bool = False, caps: Optional[Tuple[int, int]] = None):
    """O8e on a subgraph in local ids; returns (side, coarsening levels)."""
    vw, ew = _weights(sub)
    side = np.zeros(max(sub.n, 1), np.uint8)
    nlev = ctypes.c_int32(0)
    rc = _load().or_ml_bipartition(sub.n, _p(_i32(sub.xadj)), _p(_i32(sub.adjncy)), _p(ew), _p(vw), level, first,
                                   f, lk_, seed, _p(side, PU8), int(fm_passes), int(pool),
                                   -1 if caps is None else caps[0], -1 if caps is None else caps[1],
                                   ctypes.byref(nlev))
    if rc != 0:
        raise RuntimeError(f"oracle ml_bipartition failed: {rc}")
    return side[:sub.n], int(nlev.value)


FM_STALL = 64


def fm2(sub, side, cap0: int, cap1: int, passes: int, stall: int = FM_STALL):
    """O8b on a subgraph in local ids from the bipartition `side` (0/1);
    returns (refined side, total cut decrease)."""
    vw, ew = _weights(sub)
    sd = np.ascontiguousarray(side, dtype=np.uint8).copy()
    if sd.shape[0] == 0:
        sd = np.zeros(1, np.uint8)
    dec = ctypes.c_int64(0)
    rc = _load().or_fm2_stall(sub.n, _p(_i32(sub.xadj)), _p(_i32(sub.adjncy)), _p(ew), _p(vw), _p(sd, PU8),
                              cap0, cap1, passes, stall, ctypes.byref(dec))
    if rc != 0:
        raise RuntimeError(f"oracle fm2 failed: {rc}")
    return sd[:sub.n], int(dec.value)


def eps_root(x: int, r: int) -> int:
    """O8d: the largest q with P_r(q) <= x (2^32-scaled r-th root of x / 2^32)."""
    return int(_load().or_eps_root(x, r))


def adaptive_caps(cV: int, k: int, eps: float, cB: int, f: int) -> Tuple[int, int]:
    """O8d: caps of the two sides of a block of weight cB and final count f."""
    c0, c1 = ctypes.c_int64(0), ctypes.c_int64(0)
    _load().or_adaptive_caps(cV, k, eps_ppm(eps), cB, f, ctypes.byref(c0), ctypes.byref(c1))
    return int(c0.value), int(c1.value)


def rg_cmp(d1: int, c1: int, d2: int, c2: int) -> int:
    return int(_load().or_rg_cmp(d1, c1, d2, c2))


def set_visit_order(mode: int) -> None:
    _load().or_set_visit_order(mode)


def sub_class(seed: int, level: int, v: int) -> int:
    return int(_load().or_sub_class(seed & (2**64 - 1), level, v))


def lp_subround(g, level: int, r: int, s: int, tag: int, seed: int, label, wt, capv=None, caps: int = 0,
                active=None, fav=None):
    """One O3 sub-round from an arbitrary state.  Returns (label, wt, fav, moved, nmoved)."""
    vw, ew = _weights(g)
    n = g.n
    label = _i32(label).copy()
    wt = np.ascontiguousarray(wt, dtype=np.int64).copy()
    favv = None if fav is None else np.ascontiguousarray(fav, dtype=np.uint32).copy()
    capv = None if capv is None else np.ascontiguousarray(capv, dtype=np.int64)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    moved = np.zeros(max(n, 1), np.uint8)
    nm = _load().or_step_lp_subround(n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), level, r, s, tag,
                                     seed, _p(label), _p(wt, P64), int(wt.shape[0]), _p(capv, P64), caps,
                                     _p(act, PU8), _p(favv, PU32), _p(moved, PU8))
    return label, wt, favv, moved[:n], int(nm)


def balance(g, level: int, seed: int, part, wt, cap):
    vw, ew = _weights(g)
    part = _i32(part).copy()
    wt = np.ascontiguousarray(wt, dtype=np.int64).copy()
    cap = np.ascontiguousarray(cap, dtype=np.int64)
    rounds = _load().or_step_balance(g.n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), level, seed,
                                     _p(part), _p(wt, P64), int(wt.shape[0]), _p(cap, P64))
    return part, wt, int(rounds)


def balance_pq(g, level: int, seed: int, part, wt, cap):
    vw, ew = _weights(g)
    part = _i32(part).copy()
    wt = np.ascontiguousarray(wt, dtype=np.int64).copy()
    cap = np.ascontiguousarray(cap, dtype=np.int64)
    rounds = _load().or_step_balance_pq(g.n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(vw), _p(ew), level, seed,
                                     _p(part), _p(wt, P64), int(wt.shape[0]), _p(cap, P64))
    return part, wt, int(rounds)


def cut(g, part) -> int:
    ew = None if g.adjwgt is None else _i32(g.adjwgt)
    return int(_load().or_step_cut(g.n, _p(_i32(g.xadj)), _p(_i32(g.adjncy)), _p(ew), _p(_i32(part))))


def count_labels(label) -> int:
    label = _i32(label)
    return int(_load().or_count_labels(label.shape[0], _p(label)))
