"""Seeded synthetic graph generators (inputs only).

Stand-ins for the benchmark families the paper evaluates on (Section 6,
"Instances": meshes, random geometric graphs, skewed social/web graphs):

* ``grid(rows, cols)``      - 2D 5-point grid, id = row*cols + col
* ``rgg(n, avgdeg, seed)``  - 2D random geometric graph, ids sorted by cell
* ``rmat(scale, nedges, seed)`` - symmetrised RMAT (0.57, 0.19, 0.19, 0.05)
* ``random_graph(...)``     - small weighted random graphs for tests

Graphs are symmetric CSR with int32 arrays; neighbours ascending; no self
loops or duplicates.  This module holds none of the partitioner's arithmetic:
both the HIP path and the CPU oracle consume what it makes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libkmpgen.so")


def build(force: bool = True) -> str:
    """Compile the generator library in-tree with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _KG(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("xadj", ctypes.POINTER(ctypes.c_int32)),
                ("adjncy", ctypes.POINTER(ctypes.c_int32)),
                ("maxdeg", ctypes.c_int32), ("nisolated", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.kg_grid.restype = ctypes.POINTER(_KG)
        lib.kg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32]
        lib.kg_rgg.restype = ctypes.POINTER(_KG)
        lib.kg_rgg.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64]
        lib.kg_rmat.restype = ctypes.POINTER(_KG)
        lib.kg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_uint64]
        lib.kg_free.argtypes = [ctypes.POINTER(_KG)]
        lib.kg_free.restype = None
        lib.kg_sm64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.kg_sm64.restype = ctypes.c_uint64
        lib.kg_rgg_radius.argtypes = [ctypes.c_int32, ctypes.c_double]
        lib.kg_rgg_radius.restype = ctypes.c_int64
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Symmetric CSR graph. ``vwgt``/``adjwgt`` None means unit weights."""
    xadj: np.ndarray
    adjncy: np.ndarray
    vwgt: Optional[np.ndarray] = None
    adjwgt: Optional[np.ndarray] = None
    name: str = ""
    maxdeg: int = 0
    nisolated: int = 0

    @property
    def n(self) -> int:
        return int(self.xadj.shape[0]) - 1

    @property
    def m(self) -> int:
        """Directed adjacency entries (= 2 x undirected edges)."""
        return int(self.xadj[-1])


def _take(ptr, name: str) -> Graph:
    if not ptr:
        raise MemoryError("graph generator failed: " + name)
    g = ptr.contents
    n, m = g.n, g.m
    xadj = np.ctypeslib.as_array(g.xadj, shape=(n + 1,)).copy()
    adjncy = np.ctypeslib.as_array(g.adjncy, shape=(max(m, 1),))[:m].copy()
    out = Graph(xadj, adjncy, None, None, name, int(g.maxdeg), int(g.nisolated))
    _load().kg_free(ptr)
    return out


def sm64(seed: int, i: int) -> int:
    """i-th SplitMix64 draw of stream ``seed`` (counter-based)."""
    return int(_load().kg_sm64(seed & (2**64 - 1), i & (2**64 - 1)))


def grid(rows: int, cols: int) -> Graph:
    return _take(_load().kg_grid(rows, cols), f"grid{rows}x{cols}")


def rgg_radius(n: int, avgdeg: float = 8.0) -> int:
    return int(_load().kg_rgg_radius(n, avgdeg))


def rgg(n: int, avgdeg: float = 8.0, seed: int = 1) -> Graph:
    return _take(_load().kg_rgg(n, avgdeg, seed), f"rgg{n}")


def rmat(scale: int, nedges: int, seed: int = 1, abc=(57, 19, 19)) -> Graph:
    return _take(_load().kg_rmat(scale, nedges, abc[0], abc[1], abc[2], seed), f"rmat{scale}")


def random_graph(n: int, avgdeg: float, seed: int, max_vw: int = 1, max_ew: int = 1,
                 isolated_frac: float = 0.0) -> Graph:
    """Small Erdos-Renyi-like graph with optional random integer weights (tests)."""
    rng = np.random.default_rng(seed)
    if n <= 1:
        xadj = np.zeros(n + 1, np.int32)
        return Graph(xadj, np.zeros(0, np.int32),
                     None if max_vw <= 1 else rng.integers(1, max_vw + 1, n).astype(np.int32),
                     None if max_ew <= 1 else np.zeros(0, np.int32), f"rand{n}")
    ne = int(n * avgdeg / 2)
    u = rng.integers(0, n, ne)
    v = rng.integers(0, n, ne)
    if isolated_frac > 0:
        iso = rng.random(n) < isolated_frac
        keep = ~(iso[u] | iso[v])
        u, v = u[keep], v[keep]
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v).astype(np.int64)
    b = np.maximum(u, v).astype(np.int64)
    key = np.unique(a * n + b)
    a, b = key // n, key % n
    w = rng.integers(1, max_ew + 1, a.shape[0]).astype(np.int64) if max_ew > 1 else None
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    xadj = np.zeros(n + 1, np.int64)
    np.add.at(xadj, src + 1, 1)
    xadj = np.cumsum(xadj).astype(np.int32)
    adjwgt = None
    if w is not None:
        ww = np.concatenate([w, w])[order]
        adjwgt = ww.astype(np.int32)
    vwgt = rng.integers(1, max_vw + 1, n).astype(np.int32) if max_vw > 1 else None
    return Graph(xadj, dst.astype(np.int32), vwgt, adjwgt, f"rand{n}")


# ---------------------------------------------------------------------------
# Named workloads (Section 6 stand-ins).  C = 160, epsilon = 0.03 throughout.
# ---------------------------------------------------------------------------

def batch_sizes(count: int = 256, seed: int = 0x5EED_BA7C, lo: int = 10, span: int = 6):
    """n_i = floor(2^(lo + span*u_i)), u_i uniform in [0,1) from SplitMix64."""
    out = []
    for i in range(count):
        u = (sm64(seed, i) >> 11) * (1.0 / (1 << 53))
        out.append(int(math.floor(2.0 ** (lo + span * u))))
    return out


def batch_graph(i: int, n_i: int) -> Graph:
    """Graph i of the batched workload: even i grid, odd i RGG (avg degree 8)."""
    if i % 2 == 0:
        a = max(1, int(math.isqrt(n_i)))
        return grid(a, n_i // a)
    return rgg(n_i, 8.0, seed=i)


SERVING_KS = (2, 8, 64, 512, 4096)


def serving_jobs(count: int = 2000, seed: int = 0x5E2F_1CE5, lo: int = 12, hi: int = 21):
    """Jobs of the serving workload: job j has type uniform over (grid, rgg, rmat), n log-uniform in
    [2^lo, 2^hi], k uniform over SERVING_KS, eps 0.03 and seed j (draws from SplitMix64)."""
    out = []
    for j in range(count):
        typ = ("grid", "rgg", "rmat")[sm64(seed, 3 * j) % 3]
        u = (sm64(seed, 3 * j + 1) >> 11) * (1.0 / (1 << 53))
        n = int(math.floor(2.0 ** (lo + (hi - lo) * u)))
        k = SERVING_KS[sm64(seed, 3 * j + 2) % len(SERVING_KS)]
        out.append((typ, n, k, j))
    return out


def serving_pool_key(typ: str, n: int, buckets: int = 12, lo: int = 12, hi: int = 21):
    """Graph of the shared pool that serves a job of this type and size: RMAT at scale round(log2 n),
    grids and RGGs at the nearest of `buckets` log-spaced sizes in [2^lo, 2^hi]."""
    if typ == "rmat":
        return ("rmat", min(hi, max(lo, int(round(math.log2(n))))))
    b = min(buckets - 1, max(0, int((math.log2(n) - lo) / (hi - lo) * buckets)))
    return (typ, int(math.floor(2.0 ** (lo + (hi - lo) * (b + 0.5) / buckets))))


def pool_graph(key) -> Graph:
    """RMAT: scale s with 8 * 2^s generated edges (edge factor 8); grid: floor(sqrt n) rows; RGG: degree 8."""
    typ, x = key
    if typ == "rmat":
        return rmat(x, 8 << x, seed=x)
    if typ == "grid":
        a = max(1, int(math.isqrt(x)))
        return grid(a, x // a)
    return rgg(x, 8.0, seed=x)


WORKLOADS = {
    "grid128": dict(k=8, eps=0.03, seed=1, desc="grid128: 2D 5-point grid 128x128, k=8, eps=0.03, seed 1"),
    "rgg20": dict(k=64, eps=0.03, seed=1,
                  desc="rgg20: 2D random geometric graph, n=2^20, avg degree 8, k=64, eps=0.03, seed 1"),
    "rmat22": dict(k=1 << 15, eps=0.03, seed=1,
                   desc="rmat22: symmetrised RMAT, n=2^22, 2^25 generated edges (0.57, 0.19, 0.19), "
                        "k=2^15, eps=0.03, seed 1"),
}


def workload(name: str) -> Graph:
    if name == "grid128":
        return grid(128, 128)
    if name == "rgg20":
        return rgg(1 << 20, 8.0, seed=1)
    if name == "rmat22":
        return rmat(22, 1 << 25, seed=1)
    if name.startswith("grid") and "x" in name:
        r, c = name[4:].split("x")
        return grid(int(r), int(c))
    if name.startswith("rgg_"):
        return rgg(int(name[4:]), 8.0, seed=1)
    if name.startswith("rmat_"):
        s = int(name[5:])
        return rmat(s, 8 << s, seed=1)
    raise KeyError(name)
