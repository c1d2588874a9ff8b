"""Independent dense-matrix helpers for pinning the oracle on small graphs.

These compute quantities straight from their definitions in linear algebra
(adjacency matrix A, indicator matrix P), not from the oracle's code paths.
"""
import itertools

import numpy as np


def dense_adj(g) -> np.ndarray:
    n = g.n
    A = np.zeros((n, n), dtype=np.int64)
    w = g.adjwgt if g.adjwgt is not None else np.ones(g.m, np.int64)
    for v in range(n):
        for e in range(g.xadj[v], g.xadj[v + 1]):
            A[v, g.adjncy[e]] += int(w[e])
    return A


def node_w(g) -> np.ndarray:
    return (np.asarray(g.vwgt, np.int64) if g.vwgt is not None else np.ones(g.n, np.int64))


def indicator(labels, ncols=None) -> np.ndarray:
    labels = np.asarray(labels, np.int64)
    k = int(labels.max()) + 1 if ncols is None else ncols
    P = np.zeros((labels.shape[0], k), dtype=np.int64)
    P[np.arange(labels.shape[0]), labels] = 1
    return P


def cut_dense(A, part) -> int:
    """Sec. 2: weight of the edges whose ends lie in different blocks."""
    part = np.asarray(part)
    diff = part[:, None] != part[None, :]
    return int((A * diff).sum() // 2)


def brute_force_min_cut(A, c, k, cap):
    """Minimum cut over all assignments to k labelled blocks with every block <= cap."""
    n = A.shape[0]
    best = None
    for assign in itertools.product(range(k), repeat=n):
        a = np.array(assign)
        bw = np.bincount(a, weights=c, minlength=k)
        if (bw > cap).any():
            continue
        cu = cut_dense(A, a)
        if best is None or cu < best:
            best = cu
    return best


def csr_from_dense(A, vwgt=None):
    from paper_2105_02022_amd.gen import Graph
    n = A.shape[0]
    xadj = [0]
    adj, w = [], []
    for v in range(n):
        for u in range(n):
            if A[v, u]:
                adj.append(u)
                w.append(int(A[v, u]))
        xadj.append(len(adj))
    aw = np.array(w, np.int32)
    return Graph(np.array(xadj, np.int32), np.array(adj, np.int32),
                 None if vwgt is None else np.asarray(vwgt, np.int32),
                 None if (aw == 1).all() else aw, "dense")


def two_cliques(s):
    A = np.zeros((2 * s, 2 * s), np.int64)
    A[:s, :s] = 1
    A[s:, s:] = 1
    np.fill_diagonal(A, 0)
    return A


def path(n):
    A = np.zeros((n, n), np.int64)
    for i in range(n - 1):
        A[i, i + 1] = A[i + 1, i] = 1
    return A


def with_hubs(g, degrees, seed):
    """`g` plus one new vertex per entry of `degrees`, each joined to that many
    distinct random vertices of `g` (unit weights; symmetric; sorted rows)."""
    from paper_2105_02022_amd.gen import Graph
    assert g.vwgt is None and g.adjwgt is None
    rng = np.random.default_rng(seed)
    n0 = g.n
    src = np.repeat(np.arange(n0, dtype=np.int64), np.diff(g.xadj))
    dst = np.asarray(g.adjncy, np.int64)
    us, vs = [src], [dst]
    for h, d in enumerate(degrees):
        nb = rng.choice(n0, size=d, replace=False).astype(np.int64)
        hub = np.full(d, n0 + h, np.int64)
        us += [hub, nb]
        vs += [nb, hub]
    u = np.concatenate(us)
    v = np.concatenate(vs)
    n = n0 + len(degrees)
    key = np.unique(u * n + v)
    u, v = key // n, key % n
    xadj = np.zeros(n + 1, np.int64)
    np.add.at(xadj, u + 1, 1)
    return Graph(np.cumsum(xadj).astype(np.int32), v.astype(np.int32), None, None, "hubs",
                 int(np.diff(np.cumsum(xadj)).max()))
