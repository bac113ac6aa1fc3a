"""Seeded synthetic graph inputs shared by the CPU oracle tests and the HIP engine.

Only input construction lives here (R-MAT, grids with random edge deletion,
random edge weights, CSR/CSC assembly, source choice); none of the graph
algorithms does.  The heavy lifting is the C library ``libsxgen.so`` built
from ``sxgen.c`` in this directory.

The workloads follow the paper's evaluation inputs (Section 6, dataset table):
R-MAT graphs stand in for its Kron/R-MAT/social graphs and 2D grids with 10%
of edges deleted for its high-diameter road maps; the real datasets are not
used.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsxgen.so")

_lib = None


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int32)),
                ("indices", ctypes.POINTER(ctypes.c_int32))]


def build(verbose: bool = False) -> str:
    """Compile libsxgen.so with gcc (OpenMP)."""
    import subprocess
    src = os.path.join(_HERE, "sxgen.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", src, "-o", tmp]
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
        L.sxg_rmat.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_CSR)]
        L.sxg_grid.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(_CSR)]
        L.sxg_free.argtypes = [ctypes.POINTER(_CSR)]
        L.sxg_weights.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        L.sxg_transpose.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.sxg_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.sxg_splitmix64_at.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """Host CSR graph.  Undirected graphs store both arcs of every edge.

    offsets: int32 [n+1]; indices: int32 [m] (rows sorted ascending);
    weights: uint32 [m] or None.  Directed graphs also carry the in-arc CSC
    (in_offsets, in_indices, in_weights)."""
    n: int
    offsets: np.ndarray
    indices: np.ndarray
    weights: Optional[np.ndarray] = None
    directed: bool = False
    in_offsets: Optional[np.ndarray] = None
    in_indices: Optional[np.ndarray] = None
    in_weights: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.indices.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64)).astype(np.int32)

    def in_degree(self) -> np.ndarray:
        if not self.directed:
            return self.out_degree()
        return np.diff(self.in_offsets.astype(np.int64)).astype(np.int32)


def _take(csr: _CSR) -> Tuple[np.ndarray, np.ndarray]:
    n, m = csr.n, csr.m
    off = np.ctypeslib.as_array(csr.offsets, shape=(n + 1,)).copy()
    idx = (np.ctypeslib.as_array(csr.indices, shape=(m,)).copy() if m > 0
           else np.zeros(0, dtype=np.int32))
    lib().sxg_free(ctypes.byref(csr))
    return off, idx


def splitmix64_at(seed: int, i: int) -> int:
    return int(lib().sxg_splitmix64_at(seed & (2**64 - 1), i & (2**64 - 1)))


def add_weights(g: Graph, lo: int, hi: int, seed: int) -> Graph:
    """Uniform integer weights in [lo, hi]; both arcs of an undirected edge share one."""
    w = np.empty(g.m, dtype=np.uint32)
    rc = lib().sxg_weights(g.n, _ptr(g.offsets), _ptr(g.indices), lo, hi, seed,
                           0 if g.directed else 1, _ptr(w))
    if rc != 0:
        raise ValueError(f"sxg_weights failed: {rc}")
    g.weights = w
    if g.directed and g.in_offsets is not None:
        _fill_csc(g)
    g.meta["weights"] = (lo, hi, seed)
    return g


def _fill_csc(g: Graph) -> None:
    ino = np.empty(g.n + 1, dtype=np.int32)
    ini = np.empty(g.m, dtype=np.int32)
    inw = np.empty(g.m, dtype=np.uint32) if g.weights is not None else None
    rc = lib().sxg_transpose(g.n, g.m, _ptr(g.offsets), _ptr(g.indices), _ptr(g.weights),
                             _ptr(ino), _ptr(ini), _ptr(inw))
    if rc != 0:
        raise ValueError(f"sxg_transpose failed: {rc}")
    g.in_offsets, g.in_indices, g.in_weights = ino, ini, inw


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, directed: bool = False, weights: Optional[Tuple[int, int]] = None,
         weight_seed: Optional[int] = None) -> Graph:
    """R-MAT graph, 2^scale vertices, edge_factor * 2^scale generated edges,
    deduplicated, self loops removed; symmetrised unless directed."""
    csr = _CSR()
    rc = lib().sxg_rmat(scale, edge_factor, a, b, c, seed, 1 if directed else 0, ctypes.byref(csr))
    if rc != 0:
        raise ValueError(f"sxg_rmat failed: {rc}")
    off, idx = _take(csr)
    g = Graph(n=1 << scale, offsets=off, indices=idx, directed=directed,
              name=f"rmat{scale}{'d' if directed else 'u'}",
              meta=dict(kind="rmat", scale=scale, edge_factor=edge_factor, abc=(a, b, c), seed=seed))
    if directed:
        _fill_csc(g)
    if weights is not None:
        add_weights(g, weights[0], weights[1], seed + 100 if weight_seed is None else weight_seed)
    return g


def grid(side: int, p_del: float = 0.1, seed: int = 203, weights: Optional[Tuple[int, int]] = None,
         weight_seed: int = 103) -> Graph:
    """side x side 4-neighbour grid (vertex id = row*side + col), each edge
    deleted independently with probability p_del."""
    csr = _CSR()
    rc = lib().sxg_grid(side, p_del, seed, ctypes.byref(csr))
    if rc != 0:
        raise ValueError(f"sxg_grid failed: {rc}")
    off, idx = _take(csr)
    g = Graph(n=side * side, offsets=off, indices=idx, directed=False, name=f"grid{side}",
              meta=dict(kind="grid", side=side, p_del=p_del, seed=seed))
    if weights is not None:
        add_weights(g, weights[0], weights[1], weight_seed)
    return g


def from_edges(n: int, edges: Sequence[Tuple[int, int]], weights: Optional[Sequence[int]] = None,
               directed: bool = False, name: str = "edges") -> Graph:
    """Small explicit graph.  Undirected edges are stored as both arcs with the
    same weight; duplicate arcs keep the smallest weight; self loops are dropped."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = (np.asarray(weights, dtype=np.int64) if weights is not None
         else np.zeros(len(e), dtype=np.int64))
    if len(e):
        if e.min() < 0 or e.max() >= n:
            raise ValueError("vertex id out of range")
    keep = e[:, 0] != e[:, 1]
    e, w = e[keep], w[keep]
    if not directed:
        e = np.concatenate([e, e[:, ::-1]])
        w = np.concatenate([w, w])
    order = np.lexsort((w, e[:, 1], e[:, 0]))
    e, w = e[order], w[order]
    if len(e):
        first = np.ones(len(e), dtype=bool)
        first[1:] = (e[1:, 0] != e[:-1, 0]) | (e[1:, 1] != e[:-1, 1])
        e, w = e[first], w[first]
    counts = np.bincount(e[:, 0], minlength=n) if len(e) else np.zeros(n, dtype=np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    g = Graph(n=n, offsets=off.astype(np.int32), indices=e[:, 1].astype(np.int32),
              weights=(w.astype(np.uint32) if weights is not None else None),
              directed=directed, name=name)
    if directed:
        _fill_csc(g)
    return g


def bp_priors(n: int, seed: int, lo: float = 0.1, hi: float = 0.9) -> np.ndarray:
    """Prior marginals P(x_v = 1) of a binary MRF over n vertices: float32,
    uniform in [lo, hi] from a seeded numpy Generator (the belief-propagation
    workloads' unary potentials)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=n).astype(np.float32)


def max_degree_vertex(g: Graph) -> int:
    """Source vertex used by the workloads: highest out-degree, ties to the lowest id."""
    if g.n == 0:
        return -1
    return int(np.argmax(g.out_degree()))


def random_graph(n: int, p: float, seed: int, directed: bool = False,
                 weights: Optional[Tuple[int, int]] = None) -> Graph:
    """Erdos-Renyi G(n, p) from a numpy Generator (small test graphs)."""
    rng = np.random.default_rng(seed)
    if directed:
        mask = rng.random((n, n)) < p
        np.fill_diagonal(mask, False)
        s, t = np.nonzero(mask)
    else:
        mask = np.triu(rng.random((n, n)) < p, 1)
        s, t = np.nonzero(mask)
    edges = np.stack([s, t], axis=1)
    w = None
    if weights is not None:
        w = rng.integers(weights[0], weights[1] + 1, size=len(edges))
    return from_edges(n, edges, w, directed=directed, name=f"er{n}")


# ---------------------------------------------------------------------------
# The evaluation workloads (seeds: graph = workload number, weights = +100,
# deletions = +200)
# ---------------------------------------------------------------------------

def workload_graph(name: str, scale_override: Optional[int] = None, side_override: Optional[int] = None) -> Graph:
    """rmat16   : BFS on undirected R-MAT scale 16
       rmat22   : BFS/SSSP/k-core on undirected R-MAT scale 22, weights [1,64]
       grid4096 : BFS/SSSP on a 4096^2 grid, 10% edges deleted, weights [1,1000]
       rmat24d  : PageRank / k-core on directed R-MAT scale 24"""
    if name == "rmat16":
        return rmat(scale_override or 16, seed=1, weights=(1, 64), weight_seed=101)
    if name == "rmat22":
        return rmat(scale_override or 22, seed=2, weights=(1, 64), weight_seed=102)
    if name == "grid4096":
        return grid(side_override or 4096, 0.1, seed=203, weights=(1, 1000), weight_seed=103)
    if name == "rmat24d":
        return rmat(scale_override or 24, seed=4, directed=True)
    raise KeyError(name)


def batch_workload(n_rmat: int = 48, n_grid: int = 16, n_queries: int = 256, scale_range=(12, 20),
                   side_range=(256, 2048), seed: int = 1000):
    """The batched workload: n_rmat undirected R-MAT graphs (edge factor 16,
    scales uniform in scale_range) and n_grid grids (sides uniform in
    side_range, 10 % of edges deleted), all with weights in [1, 64]; then
    n_queries queries with sources drawn uniformly over non-isolated vertices
    of a uniformly chosen graph, alternating BFS and SSSP.
    Graph i uses seed `seed + i`.  Returns (graphs, queries) with queries as
    (graph index, 'bfs' | 'sssp', source)."""
    rng = np.random.default_rng(seed)
    graphs = []
    for i in range(n_rmat):
        s = int(rng.integers(scale_range[0], scale_range[1] + 1))
        graphs.append(rmat(s, seed=seed + i, weights=(1, 64), weight_seed=seed + 5000 + i))
    for j in range(n_grid):
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        graphs.append(grid(side, 0.1, seed=seed + n_rmat + j, weights=(1, 64),
                           weight_seed=seed + 6000 + j))
    qrng = np.random.default_rng(7)
    queries = []
    for k in range(n_queries):
        gi = int(qrng.integers(0, len(graphs)))
        deg = graphs[gi].out_degree()
        cand = np.flatnonzero(deg > 0)
        src = int(cand[qrng.integers(0, len(cand))])
        queries.append((gi, "bfs" if k % 2 == 0 else "sssp", src))
    return graphs, queries
