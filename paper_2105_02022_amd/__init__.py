"""Python binding of libkmp (gfx950 deep multilevel graph partitioning).

Thin ctypes marshalling over the C ABI declared in ``include/kmp.h``: every
function here has the name of the C entry point it calls and only converts
arguments (torch device tensors -> device pointers, the current torch stream
-> hipStream_t).  All computation runs in the HIP kernels of ``libkmp.so``;
there is no fallback: if the library is missing, importing a function raises.

Build the library with ``python -m paper_2105_02022_amd.build`` (or
``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmp.so")

KMP_OK, KMP_IMBALANCED, KMP_EINVAL, KMP_EGRAPH, KMP_EOVERFLOW, KMP_ENOMEM, KMP_EHIP = 0, 1, -1, -2, -3, -4, -5
KMP_ETOOLARGE = -6
# limits of kmp_partition_noalloc (include/kmp.h)
NOALLOC_MAX_N, NOALLOC_MAX_M, NOALLOC_SCRATCH_BYTES = 65536, 1048576, 256 << 20
MAX_LEVELS = 64


PROF_CLASSES = ["rate_t0", "rate_t1", "rate_t2", "rate_hub", "admit", "apply", "lp_small", "active",
                "contract_rows", "contract", "two_hop", "ggg", "balance", "project", "schedule", "other"]


class KmpOptions(ctypes.Structure):
    _fields_ = [("validate", ctypes.c_int32), ("profile", ctypes.c_int32), ("profile_classes", ctypes.c_uint32),
                ("force_exact", ctypes.c_int32), ("small_level_n", ctypes.c_int32), ("plain_loads", ctypes.c_int32),
                ("fm_passes", ctypes.c_int32), ("ip_pool", ctypes.c_int32), ("adaptive_eps", ctypes.c_int32),
                ("pq_balance", ctypes.c_int32), ("async_lp", ctypes.c_int32), ("ip_multilevel", ctypes.c_int32)]


class KmpStats(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("lk", ctypes.c_int64), ("max_block_weight", ctypes.c_int64),
                ("levels", ctypes.c_int32), ("bipartitions", ctypes.c_int32), ("balance_rounds", ctypes.c_int32),
                ("lp_exact_subrounds", ctypes.c_int32), ("level_n", ctypes.c_int32 * (MAX_LEVELS + 1)),
                ("level_m", ctypes.c_int64 * (MAX_LEVELS + 1)), ("lp_cluster_moves", ctypes.c_int64),
                ("lp_refine_moves", ctypes.c_int64), ("lp_rated_edges", ctypes.c_int64),
                ("contracted_edges", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("ms_coarsen_lp", ctypes.c_double), ("ms_contract", ctypes.c_double),
                ("ms_initial", ctypes.c_double), ("ms_refine", ctypes.c_double),
                ("prof_launches", ctypes.c_int64 * 16), ("prof_ms", ctypes.c_double * 16),
                ("prof_bytes", ctypes.c_int64 * 16), ("workspace_bytes", ctypes.c_int64)]


_vp = ctypes.c_void_p
_i32, _i64, _u32, _u64, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
_P32 = ctypes.POINTER(ctypes.c_int32)
_P64 = ctypes.POINTER(ctypes.c_int64)

class KmpGraphDesc(ctypes.Structure):
    _fields_ = [("xadj", ctypes.c_void_p), ("adjncy", ctypes.c_void_p), ("vwgt", ctypes.c_void_p),
                ("adjwgt", ctypes.c_void_p), ("n", ctypes.c_int32), ("k", ctypes.c_int32), ("m", ctypes.c_int64),
                ("epsilon", ctypes.c_double), ("seed", ctypes.c_uint64), ("out_part", ctypes.c_void_p)]


class KmpJobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("levels", ctypes.c_int32), ("cut", ctypes.c_int64),
                ("max_block_weight", ctypes.c_int64), ("lk", ctypes.c_int64),
                ("level_n", ctypes.c_int32 * (MAX_LEVELS + 1))]


class KmpServerStats(ctypes.Structure):
    _fields_ = [("jobs_submitted", ctypes.c_int64), ("jobs_done", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("max_batch_jobs", ctypes.c_int64), ("queued", ctypes.c_int64), ("hbm_in_use", ctypes.c_int64),
                ("running_batches", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class KmpTuning(ctypes.Structure):
    _fields_ = [("small_level_n", ctypes.c_int32), ("tier0_deg", ctypes.c_int32), ("tier1_deg", ctypes.c_int32),
                ("tier2_deg", ctypes.c_int32), ("tier3_deg", ctypes.c_int32), ("hub_lds_slots", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class KmpAutotuneReport(ctypes.Structure):
    _fields_ = [("configs", ctypes.c_int32), ("reps", ctypes.c_int32), ("ms_start", ctypes.c_double),
                ("ms_best", ctypes.c_double)]


TUNING_FIELDS = ("small_level_n", "tier0_deg", "tier1_deg", "tier2_deg", "tier3_deg", "hub_lds_slots")


SIGNATURES = {
    "kmp_partition": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i64, _i32, _dbl, _u64, _vp, _vp]),
    "kmp_partition_ex": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i64, _i32, _dbl, _u64, _vp, _vp,
                                        ctypes.POINTER(KmpOptions), ctypes.POINTER(KmpStats)]),
    "kmp_partition_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i64, _i32, _dbl, _u64, _vp, _vp,
                                             ctypes.POINTER(KmpOptions), ctypes.POINTER(KmpStats)]),
    "kmp_partition_batch": (ctypes.c_int, [ctypes.POINTER(KmpGraphDesc), _i32, ctypes.POINTER(KmpJobResult), _vp,
                                           ctypes.POINTER(KmpOptions), ctypes.POINTER(KmpStats)]),
    "kmp_server_create": (_vp, [ctypes.c_size_t, _i32]),
    "kmp_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(KmpGraphDesc), ctypes.POINTER(ctypes.c_uint64)]),
    "kmp_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(KmpJobResult),
                                       ctypes.POINTER(ctypes.c_double)]),
    "kmp_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(KmpJobResult),
                                       ctypes.POINTER(ctypes.c_double)]),
    "kmp_server_stats_get": (ctypes.c_int, [_vp, ctypes.POINTER(KmpServerStats)]),
    "kmp_server_destroy": (None, [_vp]),
    "kmp_server_set_options": (ctypes.c_int, [_vp, ctypes.POINTER(KmpOptions)]),
    "kmp_set_tuning": (ctypes.c_int, [ctypes.POINTER(KmpTuning)]),
    "kmp_get_tuning": (ctypes.c_int, [ctypes.POINTER(KmpTuning)]),
    "kmp_autotune": (ctypes.c_int, [ctypes.POINTER(KmpGraphDesc), _i32, _vp, ctypes.POINTER(KmpTuning),
                                    ctypes.POINTER(KmpAutotuneReport)]),
    "kmp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "kmp_version": (ctypes.c_char_p, []),
    "kmp_lp_cluster": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _i64, _u64, _vp, _vp, _vp, _P64, _vp]),
    "kmp_two_hop": (_i64, [_vp, _vp, _vp, _vp, _i32, _i64, _vp, _vp, _vp, _vp]),
    "kmp_contract": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _P32, _P64, _vp, _vp, _vp, _vp, _vp]),
    "kmp_bipartition_round": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _vp, _P32, _P32, _P32, _i64, _u64,
                                             _vp]),
    "kmp_bipartition_round_ex": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _vp, _P32, _P32, _P32, _i64,
                                                _u64, _i32, _i32, _vp]),
    "kmp_balance": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _u64, _vp, _vp, _i32, _vp, _vp]),
    "kmp_balance_ex": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _u64, _vp, _vp, _i32, _vp, _i32, _vp]),
    "kmp_lp_refine": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _u64, _vp, _vp, _i32, _vp, _P64, _vp]),
    "kmp_lp_subround": (_i64, [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _u32, _u64, _vp, _vp, _i32, _vp, _i64,
                               _vp, _vp, _vp, _vp]),
    "kmp_lp_async": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _u32, _u64, _vp, _vp, _i32, _vp, _i64, _vp, _P64,
                                    _i32, _vp]),
}

_lib = None


def library() -> ctypes.CDLL:
    """Load libkmp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libkmp.so not found at {LIB_PATH}; build it with "
                              "`python -m paper_2105_02022_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libkmp takes device tensors")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_i32(*ts):
    import torch
    for t in ts:
        if t is not None and t.dtype != torch.int32:
            raise TypeError("graph arrays must be torch.int32")


def kmp_strerror(code: int) -> str:
    return library().kmp_strerror(code).decode()


def kmp_version() -> str:
    return library().kmp_version().decode()


def kmp_partition(xadj, adjncy, vwgt, adjwgt, k: int, epsilon: float = 0.03, seed: int = 1, out=None,
                  stream=None) -> Tuple[int, "torch.Tensor"]:
    """Returns (status, out_part).  Arrays are int32 device tensors."""
    import torch
    _check_i32(xadj, adjncy, vwgt, adjwgt)
    n = xadj.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=xadj.device)
    m = adjncy.numel()
    rc = library().kmp_partition(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, m, k, epsilon,
                                 seed & (2**64 - 1), _ptr(out), _stream(stream))
    return rc, out


def kmp_get_tuning() -> Dict:
    """The process-wide tuning (launch choices that never change the output)."""
    t = KmpTuning()
    rc = library().kmp_get_tuning(ctypes.byref(t))
    if rc != KMP_OK:
        raise RuntimeError(kmp_strerror(rc))
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def kmp_set_tuning(tuning: Optional[Dict] = None) -> int:
    """Set the process-wide tuning from a dict with the TUNING_FIELDS (None: the defaults; a missing
    hub_lds_slots: its default)."""
    if tuning is None:
        return library().kmp_set_tuning(None)
    t = KmpTuning()
    for f in TUNING_FIELDS:
        setattr(t, f, int(tuning.get(f, 0) if f == "hub_lds_slots" else tuning[f]))
    return library().kmp_set_tuning(ctypes.byref(t))


def kmp_autotune(xadj, adjncy, vwgt, adjwgt, k: int, epsilon: float = 0.03, seed: int = 1, out=None,
                 reps: int = 3, stream=None) -> Tuple[int, Dict, Dict]:
    """Time kmp_partition on this job under candidate tunings and keep the fastest (process-wide).
    Returns (status, chosen tuning, report)."""
    import torch
    n = xadj.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=xadj.device)
    d = KmpGraphDesc()
    _fill_desc(d, dict(xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, out=out, k=k, epsilon=epsilon,
                       seed=seed))
    t, r = KmpTuning(), KmpAutotuneReport()
    rc = library().kmp_autotune(ctypes.byref(d), int(reps), _stream(stream), ctypes.byref(t), ctypes.byref(r))
    return rc, {f: getattr(t, f) for f in TUNING_FIELDS}, {f[0]: getattr(r, f[0]) for f in r._fields_}


def kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k: int, epsilon: float = 0.03, seed: int = 1, out=None,
                     stream=None, validate: bool = False, profile: bool = False,
                     profile_classes=None, force_exact: bool = False,
                     small_level_n: int = 0, plain_loads: bool = False,
                     fm_passes: int = 0, ip_pool: bool = False,
                     adaptive_eps: bool = False, pq_balance: bool = False,
                     async_lp: int = 0, ip_multilevel: bool = False) -> Tuple[int, "torch.Tensor", Dict]:
    """Returns (status, out_part, stats dict).  `profile_classes`: names from PROF_CLASSES to time
    (None: all).  `force_exact`: contended LP sub-rounds take the host-synchronised exact path.
    `small_level_n`: largest level run by the one-workgroup LP (0 default, -1 never).
    `plain_loads`: the lane rating kernel gathers with plain loads (the buffer-load path is the default).
    `fm_passes`: 2-way FM passes after every greedy growth (0..16; 0 = none).
    `ip_pool`: the initial bipartitioning also runs BFS and random growths.
    `adaptive_eps`: bipartitions bound their sides by the adaptive imbalance (paper Sec. 2, Alg. 2).
    `pq_balance`: the queue balancer of paper Sec. 5.3 instead of sorted rounds.
    `async_lp`: 1 = asynchronous LP (paper Sec. 5.1 / 5.3), 2 = the same one node per launch (tests).
    `ip_multilevel`: multilevel initial bipartitioning (paper Sec. 5.2)."""
    import torch
    _check_i32(xadj, adjncy, vwgt, adjwgt)
    n = xadj.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=xadj.device)
    opt = KmpOptions()
    opt.validate = int(validate)
    opt.profile = int(profile)
    opt.force_exact = int(force_exact)
    opt.small_level_n = int(small_level_n)
    opt.plain_loads = int(plain_loads)
    opt.fm_passes = int(fm_passes)
    opt.ip_pool = int(ip_pool)
    opt.adaptive_eps = int(adaptive_eps)
    opt.pq_balance = int(pq_balance)
    opt.async_lp = int(async_lp)
    opt.ip_multilevel = int(ip_multilevel)
    if profile_classes:
        opt.profile_classes = sum(1 << PROF_CLASSES.index(c) for c in profile_classes)
    st = KmpStats()
    rc = library().kmp_partition_ex(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, adjncy.numel(), k,
                                    epsilon, seed & (2**64 - 1), _ptr(out), _stream(stream), ctypes.byref(opt),
                                    ctypes.byref(st))
    stats = _stats_dict(st, profile)
    return rc, out, stats


def kmp_partition_noalloc(xadj, adjncy, vwgt, adjwgt, k: int, epsilon: float = 0.03, seed: int = 1, out=None,
                          stream=None, validate: bool = False, force_exact: bool = False, small_level_n: int = 0,
                          fm_passes: int = 0, ip_pool: bool = False,
                          adaptive_eps: bool = False, pq_balance: bool = False,
                          async_lp: int = 0, ip_multilevel: bool = False) -> Tuple[int, "torch.Tensor", Dict]:
    """kmp_partition_noalloc: as kmp_partition_ex, with every device buffer inside the library's fixed
    scratch region (n <= NOALLOC_MAX_N, m <= NOALLOC_MAX_M, else KMP_ETOOLARGE).  `out` should be
    given by callers that must not allocate."""
    import torch
    _check_i32(xadj, adjncy, vwgt, adjwgt)
    n = xadj.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=xadj.device)
    opt = KmpOptions()
    opt.validate = int(validate)
    opt.force_exact = int(force_exact)
    opt.small_level_n = int(small_level_n)
    opt.fm_passes = int(fm_passes)
    opt.ip_pool = int(ip_pool)
    opt.adaptive_eps = int(adaptive_eps)
    opt.pq_balance = int(pq_balance)
    opt.async_lp = int(async_lp)
    opt.ip_multilevel = int(ip_multilevel)
    st = KmpStats()
    rc = library().kmp_partition_noalloc(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, adjncy.numel(), k,
                                         epsilon, seed & (2**64 - 1), _ptr(out), _stream(stream),
                                         ctypes.byref(opt), ctypes.byref(st))
    return rc, out, _stats_dict(st, False)


def _stats_dict(st: "KmpStats", profile: bool) -> Dict:
    L = st.levels
    stats = {f[0]: getattr(st, f[0]) for f in KmpStats._fields_
             if not f[0].startswith(("reserved", "prof_", "level_"))}
    stats["level_n"] = list(st.level_n[:L + 1])
    stats["level_m"] = list(st.level_m[:L + 1])
    if profile:
        stats["prof"] = {name: {"launches": st.prof_launches[i], "ms": st.prof_ms[i], "bytes": st.prof_bytes[i]}
                         for i, name in enumerate(PROF_CLASSES)}
    return stats


def kmp_partition_batch(jobs, stream=None, validate: bool = False, profile: bool = False,
                        profile_classes=None, force_exact: bool = False,
                        small_level_n: int = 0, plain_loads: bool = False,
                        fm_passes: int = 0, ip_pool: bool = False,
                        adaptive_eps: bool = False, pq_balance: bool = False,
                        async_lp: int = 0, ip_multilevel: bool = False) -> Tuple[int, List[Dict], Dict]:
    """Partition many graphs in one pass.  `jobs`: sequence of dicts with device tensors
    xadj, adjncy, vwgt (or None), adjwgt (or None), out (int32 [n]) and k, epsilon, seed.
    Returns (call status, per-job result dicts, aggregate stats)."""
    descs = (KmpGraphDesc * max(len(jobs), 1))()
    for i, j in enumerate(jobs):
        _fill_desc(descs[i], j)
    res = (KmpJobResult * max(len(jobs), 1))()
    opt = KmpOptions()
    opt.validate = int(validate)
    opt.profile = int(profile)
    opt.force_exact = int(force_exact)
    opt.small_level_n = int(small_level_n)
    opt.plain_loads = int(plain_loads)
    opt.fm_passes = int(fm_passes)
    opt.ip_pool = int(ip_pool)
    opt.adaptive_eps = int(adaptive_eps)
    opt.pq_balance = int(pq_balance)
    opt.async_lp = int(async_lp)
    opt.ip_multilevel = int(ip_multilevel)
    if profile_classes:
        opt.profile_classes = sum(1 << PROF_CLASSES.index(c) for c in profile_classes)
    st = KmpStats()
    rc = library().kmp_partition_batch(descs, len(jobs), res, _stream(stream), ctypes.byref(opt), ctypes.byref(st))
    return rc, [_result_dict(res[i]) for i in range(len(jobs))], _stats_dict(st, profile)


def _fill_desc(d: "KmpGraphDesc", j: Dict):
    _check_i32(*[j.get(f) for f in ("xadj", "adjncy", "vwgt", "adjwgt", "out")])
    d.xadj, d.adjncy = _ptr(j["xadj"]), _ptr(j["adjncy"])
    d.vwgt, d.adjwgt = _ptr(j.get("vwgt")), _ptr(j.get("adjwgt"))
    d.n = j["xadj"].numel() - 1
    d.m = j["adjncy"].numel()
    d.k = int(j["k"])
    d.epsilon = float(j.get("epsilon", 0.03))
    d.seed = int(j.get("seed", 1)) & (2**64 - 1)
    d.out_part = _ptr(j["out"])


def _result_dict(r: "KmpJobResult") -> Dict:
    return {"status": r.status, "levels": r.levels, "cut": r.cut, "max_block_weight": r.max_block_weight,
            "lk": r.lk, "level_n": list(r.level_n[:max(r.levels, 0) + 1])}


class Server:
    """kmp_server_*: jobs submitted over time, partitioned in continuous batches by `workers` threads
    (one HIP stream each) under an HBM footprint budget.  A job is a dict as for kmp_partition_batch;
    its tensors are kept referenced here until its result is taken."""

    def __init__(self, hbm_budget_bytes: int, workers: int = 2):
        self._h = library().kmp_server_create(int(hbm_budget_bytes), int(workers))
        if not self._h:
            raise RuntimeError("kmp_server_create failed")
        self._live = {}

    def submit(self, job: Dict) -> int:
        d = KmpGraphDesc()
        _fill_desc(d, job)
        jid = ctypes.c_uint64(0)
        rc = library().kmp_server_submit(self._h, ctypes.byref(d), ctypes.byref(jid))
        if rc != KMP_OK:
            raise RuntimeError(f"kmp_server_submit: {kmp_strerror(rc)}")
        self._live[jid.value] = job
        return jid.value

    def _take(self, fn, jid: int):
        r = KmpJobResult()
        lat = ctypes.c_double(0.0)
        rc = fn(self._h, jid, ctypes.byref(r), ctypes.byref(lat))
        if rc < 0:
            raise KeyError(jid)
        if rc == 0:
            return None
        self._live.pop(jid, None)
        out = _result_dict(r)
        out["latency_ms"] = lat.value
        return out

    def set_options(self, fm_passes: int = 0, ip_pool: bool = False, adaptive_eps: bool = False,
                    pq_balance: bool = False, async_lp: int = 0, ip_multilevel: bool = False) -> int:
        """Options for jobs submitted from now on (kmp_server_set_options)."""
        o = KmpOptions()
        o.fm_passes = int(fm_passes)
        o.ip_pool = int(ip_pool)
        o.adaptive_eps = int(adaptive_eps)
        o.pq_balance = int(pq_balance)
        o.async_lp = int(async_lp)
        o.ip_multilevel = int(ip_multilevel)
        return library().kmp_server_set_options(self._h, ctypes.byref(o))

    def poll(self, jid: int) -> Optional[Dict]:
        return self._take(library().kmp_server_poll, jid)

    def wait(self, jid: int) -> Dict:
        return self._take(library().kmp_server_wait, jid)

    def stats(self) -> Dict:
        st = KmpServerStats()
        library().kmp_server_stats_get(self._h, ctypes.byref(st))
        return {f[0]: getattr(st, f[0]) for f in KmpServerStats._fields_ if f[0] != "reserved"}

    def close(self):
        if self._h:
            library().kmp_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def kmp_lp_cluster(xadj, adjncy, vwgt, adjwgt, level: int, U: int, seed: int, stream=None):
    """Returns (rounds, label, cw, fav, moves[5])."""
    import torch
    _check_i32(xadj, adjncy, vwgt, adjwgt)
    n = xadj.numel() - 1
    dev = xadj.device
    label = torch.empty(n, dtype=torch.int32, device=dev)
    cw = torch.empty(n, dtype=torch.int64, device=dev)
    fav = torch.empty(n, dtype=torch.int32, device=dev)
    moves = (ctypes.c_int64 * 5)()
    r = library().kmp_lp_cluster(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, level, U,
                                 seed & (2**64 - 1), _ptr(label), _ptr(cw), _ptr(fav),
                                 ctypes.cast(moves, _P64), _stream(stream))
    return r, label, cw, fav, list(moves)


def kmp_two_hop(xadj, adjncy, vwgt, adjwgt, U: int, label, cw, fav, stream=None) -> int:
    """In place on label (int32) and cw (int64); fav is int32 (bit pattern of uint32)."""
    _check_i32(xadj, adjncy, vwgt, adjwgt, label, fav)
    n = xadj.numel() - 1
    return library().kmp_two_hop(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, U, _ptr(label), _ptr(cw),
                                 _ptr(fav), _stream(stream))


def kmp_contract(xadj, adjncy, vwgt, adjwgt, label, stream=None):
    """Returns (status, map, cxadj, cadjncy, cvwgt, cadjwgt) trimmed to the coarse sizes."""
    import torch
    _check_i32(xadj, adjncy, vwgt, adjwgt, label)
    n = xadj.numel() - 1
    m = adjncy.numel()
    dev = xadj.device
    mp = torch.empty(n, dtype=torch.int32, device=dev)
    cx = torch.empty(n + 1, dtype=torch.int32, device=dev)
    ca = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    cv = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    cw = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    cn = ctypes.c_int32(0)
    cm = ctypes.c_int64(0)
    rc = library().kmp_contract(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, _ptr(label), _ptr(mp),
                                ctypes.byref(cn), ctypes.byref(cm), _ptr(cx), _ptr(ca), _ptr(cv), _ptr(cw),
                                _stream(stream))
    c_n, c_m = cn.value, cm.value
    return rc, mp, cx[:c_n + 1], ca[:c_m], cv[:c_n], cw[:c_m]


def kmp_bipartition_round(xadj, adjncy, vwgt, adjwgt, level: int, part, first: Sequence[int],
                          fcount: Sequence[int], lk: int, seed: int, stream=None, fm_passes: int = 0,
                          ip_pool: int = 0):
    """part updated in place; returns (status, first, fcount) as lists.  fm_passes or ip_pool
    calls kmp_bipartition_round_ex (2-way FM after every growth; BFS and random growths)."""
    _check_i32(xadj, adjncy, vwgt, adjwgt, part)
    n = xadj.numel() - 1
    nb = len(first)
    fa = (ctypes.c_int32 * (2 * nb + 1))(*first)
    fc = (ctypes.c_int32 * (2 * nb + 1))(*fcount)
    nbl = ctypes.c_int32(nb)
    if fm_passes or ip_pool:
        rc = library().kmp_bipartition_round_ex(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, level,
                                                _ptr(part), ctypes.byref(nbl), ctypes.cast(fa, _P32),
                                                ctypes.cast(fc, _P32), lk, seed & (2**64 - 1), int(fm_passes),
                                                int(ip_pool), _stream(stream))
    else:
        rc = library().kmp_bipartition_round(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, level,
                                             _ptr(part), ctypes.byref(nbl), ctypes.cast(fa, _P32),
                                             ctypes.cast(fc, _P32), lk, seed & (2**64 - 1), _stream(stream))
    q = nbl.value
    return rc, list(fa[:q]), list(fc[:q])


def kmp_balance(xadj, adjncy, vwgt, adjwgt, level: int, seed: int, part, wt, cap, stream=None) -> int:
    _check_i32(xadj, adjncy, vwgt, adjwgt, part)
    n = xadj.numel() - 1
    return library().kmp_balance(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, level, seed & (2**64 - 1),
                                 _ptr(part), _ptr(wt), wt.numel(), _ptr(cap), _stream(stream))


def kmp_balance_ex(xadj, adjncy, vwgt, adjwgt, level: int, seed: int, part, wt, cap, pq: bool = False,
                   stream=None) -> int:
    """kmp_balance_ex: pq selects the queue balancer (paper Sec. 5.3 queues)."""
    _check_i32(xadj, adjncy, vwgt, adjwgt, part)
    n = xadj.numel() - 1
    return library().kmp_balance_ex(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, level,
                                    seed & (2**64 - 1), _ptr(part), _ptr(wt), wt.numel(), _ptr(cap), int(pq),
                                    _stream(stream))


def kmp_lp_refine(xadj, adjncy, vwgt, adjwgt, level: int, seed: int, part, wt, cap, stream=None):
    _check_i32(xadj, adjncy, vwgt, adjwgt, part)
    n = xadj.numel() - 1
    moves = (ctypes.c_int64 * 5)()
    r = library().kmp_lp_refine(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, level, seed & (2**64 - 1),
                                _ptr(part), _ptr(wt), wt.numel(), _ptr(cap), ctypes.cast(moves, _P64),
                                _stream(stream))
    return r, list(moves)


def kmp_lp_subround(xadj, adjncy, vwgt, adjwgt, level: int, round_: int, s: int, tag: int, seed: int, label, wt,
                    cap_vec=None, cap_scalar: int = 0, active=None, fav=None, moved=None, stream=None) -> int:
    _check_i32(xadj, adjncy, vwgt, adjwgt, label)
    n = xadj.numel() - 1
    return library().kmp_lp_subround(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, level, round_, s, tag,
                                     seed & (2**64 - 1), _ptr(label), _ptr(wt), wt.numel(), _ptr(cap_vec),
                                     cap_scalar, _ptr(active), _ptr(fav), _ptr(moved), _stream(stream))


def kmp_lp_async(xadj, adjncy, vwgt, adjwgt, level: int, tag: int, seed: int, label, wt, cap_vec=None,
                 cap_scalar: int = 0, fav=None, serial: bool = False, stream=None):
    """kmp_lp_async: a whole asynchronous LP call (tag 2 clustering, 3 refinement); returns (rounds or error,
    moves per round)."""
    _check_i32(xadj, adjncy, vwgt, adjwgt, label)
    n = xadj.numel() - 1
    moves = (ctypes.c_int64 * 5)()
    r = library().kmp_lp_async(_ptr(xadj), _ptr(adjncy), _ptr(vwgt), _ptr(adjwgt), n, level, tag,
                               seed & (2**64 - 1), _ptr(label), _ptr(wt), wt.numel(), _ptr(cap_vec), cap_scalar,
                               _ptr(fav), ctypes.cast(moves, _P64), int(serial), _stream(stream))
    return r, list(moves)


def to_device(g, device="cuda"):
    """Copy a generator Graph (numpy CSR) to int32 device tensors."""
    import torch

    def t(a):
        return None if a is None else torch.from_numpy(a.astype("int32", copy=False)).to(device)
    return t(g.xadj), t(g.adjncy), t(g.vwgt), t(g.adjwgt)


def partition(g, k: int, epsilon: float = 0.03, seed: int = 1, device="cuda", validate: bool = False,
              fm_passes: int = 0, ip_pool: bool = False, adaptive_eps: bool = False, ip_multilevel: bool = False):
    """Convenience: partition a generator Graph; returns (status, part numpy, stats)."""
    xadj, adjncy, vwgt, adjwgt = to_device(g, device)
    rc, out, stats = kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, k, epsilon, seed, validate=validate,
                                      fm_passes=fm_passes, ip_pool=ip_pool, adaptive_eps=adaptive_eps,
                                      ip_multilevel=ip_multilevel)
    return rc, out.cpu().numpy(), stats
