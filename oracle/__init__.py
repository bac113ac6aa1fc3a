"""CPU oracle for the ACC graph engine — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The engine in ``paper_1812_04070_amd``
never does; it shares no code with it.

Serial, plain implementations (``oracle.c``) of what the paper's method
computes: queue BFS, Dijkstra / worklist Bellman-Ford / synchronous rounds for
SSSP, Batagelj-Zaversnik and naive peeling for the k-core decomposition, fp64
PageRank, fp64 belief propagation on a binary pairwise MRF; plus (``mlp.py``) the fp64 forward and backward pass of the policy
network.  Each function cites the paper passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
INF = 0xFFFFFFFF
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle (serial C, -O2, one thread)."""
    src = os.path.join(_HERE, "oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        for name, args in [("sxo_bfs", [ctypes.c_int32, vp, vp, ctypes.c_int32, vp]),
                           ("sxo_dijkstra", [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp]),
                           ("sxo_bellman_ford", [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp]),
                           ("sxo_sssp_rounds", [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, ctypes.c_int32]),
                           ("sxo_kcore_bz", [ctypes.c_int32, vp, vp, vp, vp, vp]),
                           ("sxo_kcore_peel", [ctypes.c_int32, vp, vp, vp, vp, vp]),
                           ("sxo_kcore_member", [ctypes.c_int32, vp, vp, vp, vp, ctypes.c_int32, vp]),
                           ("sxo_wcc", [ctypes.c_int32, vp, vp, vp]),
                           ("sxo_pagerank", [ctypes.c_int32, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp]),
                           ("sxo_bp", [ctypes.c_int32, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp]),
                           ("sxo_pagerank_fixpoint", [ctypes.c_int32, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                                      ctypes.c_int32, vp])]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"{what} failed with code {rc}")
    return rc


def bfs(n, offsets, indices, src):
    """Depth of every vertex from ``src`` (-1 unreachable), FIFO queue BFS."""
    off, idx = _c(offsets, np.int32), _c(indices, np.int32)
    out = np.empty(n, dtype=np.int32)
    _check(lib().sxo_bfs(n, _p(off), _p(idx), src, _p(out)), "bfs")
    return out


def sssp_dijkstra(n, offsets, indices, weights, src):
    off, idx, w = _c(offsets, np.int32), _c(indices, np.int32), _c(weights, np.uint32)
    out = np.empty(n, dtype=np.uint32)
    _check(lib().sxo_dijkstra(n, _p(off), _p(idx), _p(w), src, _p(out)), "dijkstra")
    return out


def sssp_bellman_ford(n, offsets, indices, weights, src):
    off, idx, w = _c(offsets, np.int32), _c(indices, np.int32), _c(weights, np.uint32)
    out = np.empty(n, dtype=np.uint32)
    _check(lib().sxo_bellman_ford(n, _p(off), _p(idx), _p(w), src, _p(out)), "bellman_ford")
    return out


def sssp_rounds(n, offsets, indices, weights, src, max_rounds=-1):
    """Synchronous frontier rounds; returns (dist, update_round, rounds)."""
    off, idx, w = _c(offsets, np.int32), _c(indices, np.int32), _c(weights, np.uint32)
    dist = np.empty(n, dtype=np.uint32)
    upd = np.empty(n, dtype=np.int32)
    r = _check(lib().sxo_sssp_rounds(n, _p(off), _p(idx), _p(w), src, _p(dist), _p(upd), max_rounds),
               "sssp_rounds")
    return dist, upd, r


def kcore_bz(n, offsets, indices, in_offsets=None, in_indices=None):
    off, idx = _c(offsets, np.int32), _c(indices, np.int32)
    ino, ini = _c(in_offsets, np.int32), _c(in_indices, np.int32)
    out = np.empty(n, dtype=np.int32)
    _check(lib().sxo_kcore_bz(n, _p(off), _p(idx), _p(ino), _p(ini), _p(out)), "kcore_bz")
    return out


def kcore_peel(n, offsets, indices, in_offsets=None, in_indices=None):
    off, idx = _c(offsets, np.int32), _c(indices, np.int32)
    ino, ini = _c(in_offsets, np.int32), _c(in_indices, np.int32)
    out = np.empty(n, dtype=np.int32)
    _check(lib().sxo_kcore_peel(n, _p(off), _p(idx), _p(ino), _p(ini), _p(out)), "kcore_peel")
    return out


def kcore_member(n, offsets, indices, k, in_offsets=None, in_indices=None):
    """1 where the vertex lies in the k-core (Section 6), else 0."""
    off, idx = _c(offsets, np.int32), _c(indices, np.int32)
    ino, ini = _c(in_offsets, np.int32), _c(in_indices, np.int32)
    out = np.empty(n, dtype=np.int32)
    _check(lib().sxo_kcore_member(n, _p(off), _p(idx), _p(ino), _p(ini), int(k), _p(out)), "kcore_member")
    return out


def wcc(n, offsets, indices):
    """Smallest vertex id of each vertex's connected component (union-find)."""
    off, idx = _c(offsets, np.int32), _c(indices, np.int32)
    out = np.empty(n, dtype=np.int32)
    _check(lib().sxo_wcc(n, _p(off), _p(idx), _p(out)), "wcc")
    return out


def pagerank(n, offsets, in_offsets, in_indices, d=0.85, iters=20):
    off = _c(offsets, np.int32)
    ino, ini = _c(in_offsets, np.int32), _c(in_indices, np.int32)
    out = np.empty(n, dtype=np.float64)
    _check(lib().sxo_pagerank(n, _p(off), _p(ino), _p(ini), d, iters, _p(out)), "pagerank")
    return out


# Convenience wrappers over a host Graph (anything with n/offsets/indices/...)

def bfs_g(g, src):
    return bfs(g.n, g.offsets, g.indices, src)


def sssp_g(g, src):
    return sssp_dijkstra(g.n, g.offsets, g.indices, g.weights, src)


def kcore_g(g):
    if g.directed:
        return kcore_bz(g.n, g.offsets, g.indices, g.in_offsets, g.in_indices)
    return kcore_bz(g.n, g.offsets, g.indices)


def kcore_member_g(g, k):
    if g.directed:
        return kcore_member(g.n, g.offsets, g.indices, k, g.in_offsets, g.in_indices)
    return kcore_member(g.n, g.offsets, g.indices, k)


def wcc_g(g):
    """Weak components: a directed graph's arcs are taken without direction."""
    if g.directed:
        # union of the out- and in-rows as one undirected arc list
        src = np.concatenate([np.repeat(np.arange(g.n), np.diff(g.offsets)),
                              np.repeat(np.arange(g.n), np.diff(g.in_offsets))])
        dst = np.concatenate([g.indices, g.in_indices])
        order = np.argsort(src, kind="stable")
        o = np.zeros(g.n + 1, dtype=np.int64)
        np.add.at(o, src + 1, 1)
        return wcc(g.n, np.cumsum(o), dst[order])
    return wcc(g.n, g.offsets, g.indices)


def pagerank_g(g, d=0.85, iters=20):
    if g.directed:
        return pagerank(g.n, g.offsets, g.in_offsets, g.in_indices, d, iters)
    return pagerank(g.n, g.offsets, g.offsets, g.indices, d, iters)


def bp(n, offsets, indices, weights, prior, kappa=0.5, iters=10):
    """Belief propagation (Section 6, sum-product on a binary pairwise MRF;
    Section 3.2, all vertices active, updates summed): b(v, 1) after `iters`
    synchronous iterations from the priors, fp64 (see sxo_bp in oracle.c for
    the potentials)."""
    off = _c(offsets, np.int32)
    idx = _c(indices, np.int32)
    w = _c(weights, np.uint32)
    pr = _c(prior, np.float64)
    out = np.empty(max(n, 1), dtype=np.float64)
    _check(lib().sxo_bp(n, _p(off), _p(idx), _p(w), _p(pr), float(kappa), int(iters), _p(out)), "sxo_bp")
    return out[:n]


def bp_g(g, prior, kappa=0.5, iters=10):
    if g.directed:
        raise ValueError("belief propagation runs on undirected graphs")
    return bp(g.n, g.offsets, g.indices, g.weights, prior, kappa, iters)


def pagerank_fixpoint(n, offsets, in_offsets, in_indices, d=0.85, tol=1e-14, max_iters=10000):
    """PageRank iterated to its fixed point (Section 6: until the ranks are
    stable): the fp64 recurrence of pagerank() until one step changes the
    vector by at most `tol` in L1.  Returns (ranks, steps)."""
    off = _c(offsets, np.int32)
    io = _c(in_offsets, np.int32)
    ii = _c(in_indices, np.int32)
    out = np.empty(max(n, 1), dtype=np.float64)
    steps = _check(lib().sxo_pagerank_fixpoint(n, _p(off), _p(io), _p(ii), float(d), float(tol), int(max_iters),
                                               _p(out)), "sxo_pagerank_fixpoint")
    return out[:n], steps


def pagerank_fixpoint_g(g, d=0.85, tol=1e-14, max_iters=10000):
    if g.directed:
        return pagerank_fixpoint(g.n, g.offsets, g.in_offsets, g.in_indices, d, tol, max_iters)
    return pagerank_fixpoint(g.n, g.offsets, g.offsets, g.indices, d, tol, max_iters)
