"""Generator invariants (CPU)."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np

from paper_1812_04070_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _csr_ok(g):
    off, idx = g.offsets.astype(np.int64), g.indices
    assert off[0] == 0 and off[-1] == g.m and np.all(np.diff(off) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(off))
    assert np.all(idx >= 0) and np.all(idx < g.n)
    assert not np.any(src == idx), "self loop"
    # rows strictly ascending -> sorted and no duplicates
    same_row = src[1:] == src[:-1]
    assert np.all(idx[1:][same_row] > idx[:-1][same_row])
    return src


def test_rmat_undirected_symmetric():
    g = gen.rmat(12, seed=7, weights=(1, 64))
    src = _csr_ok(g)
    key = src.astype(np.int64) * g.n + g.indices
    rkey = g.indices.astype(np.int64) * g.n + src
    order = np.argsort(key)
    assert np.array_equal(np.sort(key), np.sort(rkey))
    # weights symmetric and in range
    pos = np.searchsorted(key[order], rkey)
    assert np.array_equal(g.weights, g.weights[order][pos])
    assert g.weights.min() >= 1 and g.weights.max() <= 64
    assert g.out_degree().sum() == g.m and g.m % 2 == 0


def test_rmat_deterministic_and_thread_invariant():
    g1 = gen.rmat(13, seed=3)
    g2 = gen.rmat(13, seed=3)
    assert np.array_equal(g1.indices, g2.indices)
    code = ("import numpy as np; from paper_1812_04070_amd import gen; "
            "g = gen.rmat(13, seed=3); print(int(np.bitwise_xor.reduce(g.indices * np.arange(g.m, dtype=np.int64) % 1000003)), g.m)")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out1 = subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, env=env).decode().split()
    env["OMP_NUM_THREADS"] = "5"
    out5 = subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, env=env).decode().split()
    assert out1 == out5
    assert int(out1[1]) == g1.m
    g3 = gen.rmat(13, seed=4)
    assert g3.m != g1.m or not np.array_equal(g3.indices, g1.indices)


def test_rmat_skew():
    g = gen.rmat(14, seed=1)
    deg = g.out_degree()
    # R-MAT with a=0.57: heavy skew, many isolated vertices, hub at a low id
    assert deg.max() > 50 * deg.mean()
    assert 0.15 < (deg == 0).mean() < 0.5
    assert gen.max_degree_vertex(g) == int(np.argmax(deg))


def test_rmat_directed_csc():
    g = gen.rmat(11, seed=4, directed=True)
    src = _csr_ok(g)
    assert g.in_offsets[-1] == g.m
    # CSC is the transpose
    a = np.sort(src.astype(np.int64) * g.n + g.indices)
    isrc = np.repeat(np.arange(g.n), np.diff(g.in_offsets))
    b = np.sort(g.in_indices.astype(np.int64) * g.n + isrc)
    assert np.array_equal(a, b)


def test_grid():
    side = 128
    g = gen.grid(side, 0.1, seed=203, weights=(1, 1000))
    src = _csr_ok(g)
    assert g.out_degree().max() <= 4
    full = 2 * side * (side - 1)
    kept = g.m // 2
    assert abs((full - kept) / full - 0.1) < 0.01
    # neighbours are grid neighbours
    diff = np.abs(g.indices.astype(np.int64) - src)
    assert np.all((diff == 1) | (diff == side))
    assert g.weights.min() >= 1 and g.weights.max() <= 1000
    g0 = gen.grid(side, 0.0)
    assert g0.m == 2 * full


def test_from_edges():
    g = gen.from_edges(4, [(0, 1), (1, 0), (2, 2), (1, 3)], [5, 3, 9, 7])
    assert g.offsets.tolist() == [0, 1, 3, 3, 4]
    assert g.indices.tolist() == [1, 0, 3, 1]
    assert g.weights.tolist() == [3, 3, 7, 7]
