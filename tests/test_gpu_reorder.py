"""Parity of runs on graphs loaded with SX_REORDER (vertices renumbered by
decreasing degree inside the library): sources and results stay in the
caller's numbering, so every output must equal the oracle's on the original
graph exactly (PageRank within 1e-6 relative L1), in every arrangement."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1812_04070_amd as sx
from paper_1812_04070_amd import gen
from tests.gpu_util import announce, rel_l1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def engine():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = sx.Engine(0)
    yield e
    e.close()


GRAPHS = [
    ("er-130-dense", lambda: gen.random_graph(130, 0.3, seed=2, weights=(1, 9))),
    ("rmat12", lambda: gen.rmat(12, seed=6, weights=(1, 64))),
    ("rmat15", lambda: gen.rmat(15, seed=16, weights=(1, 64))),
    ("grid-61", lambda: gen.grid(61, 0.1, seed=7, weights=(1, 1000))),
    ("star-3000", lambda: gen.from_edges(3001, [(0, i) for i in range(1, 3001)], list(range(1, 3001)))),
    # isolated vertices and many equal degrees (ties keep id order)
    ("matching-plus-isolated", lambda: gen.from_edges(500, [(2 * i, 2 * i + 1) for i in range(200)],
                                                       [1 + i % 7 for i in range(200)])),
]

POLICIES = [
    ("auto", sx.Policy()),
    ("fused", sx.Policy(fused=sx.SX_FUSED)),
    ("unfused", sx.Policy(fused=sx.SX_UNFUSED)),
    ("pull", sx.Policy(direction=sx.SX_DIR_PULL)),
]


def _run(engine, dg, algo, src, pol):
    out, st = engine.run(dg, algo, src, pol)
    return engine.to_host(dg, algo, out), st


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_reordered_undirected(engine, name, make):
    g = make()
    src = gen.max_degree_vertex(g)
    other = int(np.flatnonzero(g.out_degree())[-1])     # a low-degree source too
    dg = engine.load(g, reorder=True)
    for s in (src, other):
        ref_d, ref_x = oracle.bfs_g(g, s), oracle.sssp_g(g, s)
        for pname, pol in POLICIES:
            announce(f"reorder {name} bfs/sssp src={s} {pname}")
            d, _ = _run(engine, dg, sx.SX_BFS, s, pol)
            np.testing.assert_array_equal(d, ref_d)
            x, _ = _run(engine, dg, sx.SX_SSSP, s, pol)
            np.testing.assert_array_equal(x, ref_x)
    ref_c = oracle.kcore_g(g)
    for pname, pol in POLICIES:
        announce(f"reorder {name} kcore {pname}")
        c, _ = _run(engine, dg, sx.SX_KCORE, -1, pol)
        np.testing.assert_array_equal(c, ref_c)
    announce(f"reorder {name} pagerank")
    r, _ = _run(engine, dg, sx.SX_PAGERANK, -1, None)
    assert rel_l1(r, oracle.pagerank_g(g)) <= 1e-6
    dg.close()


def test_reordered_directed(engine):
    g = gen.rmat(14, seed=9, directed=True)
    dg = engine.load(g, reorder=True)
    announce("reorder rmat14d pagerank")
    r, _ = _run(engine, dg, sx.SX_PAGERANK, -1, None)
    assert rel_l1(r, oracle.pagerank_g(g)) <= 1e-6
    ref_c = oracle.kcore_g(g)
    for pname, pol in POLICIES:
        announce(f"reorder rmat14d kcore {pname}")
        c, _ = _run(engine, dg, sx.SX_KCORE, -1, pol)
        np.testing.assert_array_equal(c, ref_c)
    s = gen.max_degree_vertex(g)
    announce("reorder rmat14d bfs")
    d, _ = _run(engine, dg, sx.SX_BFS, s, None)
    np.testing.assert_array_equal(d, oracle.bfs_g(g, s))
    dg.close()


def test_reordered_same_as_plain(engine):
    """The same graph loaded both ways gives the same bytes (PageRank: the
    renumbering reorders each vertex's sum, so within the tolerance)."""
    g = gen.rmat(16, seed=21, weights=(1, 64))
    a, b = engine.load(g), engine.load(g, reorder=True)
    s = gen.max_degree_vertex(g)
    for algo in (sx.SX_BFS, sx.SX_SSSP, sx.SX_KCORE):
        announce(f"reorder-vs-plain rmat16 algo={algo}")
        x, _ = _run(engine, a, algo, s if algo != sx.SX_KCORE else -1, None)
        y, _ = _run(engine, b, algo, s if algo != sx.SX_KCORE else -1, None)
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_reordered_edge_cases(engine):
    empty = gen.from_edges(0, [], [])
    announce("reorder empty graph")
    de = engine.load(empty, reorder=True)
    c, _ = _run(engine, de, sx.SX_KCORE, -1, None)
    assert c.shape == (0,)
    de.close()
    single = gen.from_edges(1, [], [])
    ds = engine.load(single, reorder=True)
    announce("reorder single vertex")
    d, _ = _run(engine, ds, sx.SX_BFS, 0, None)
    np.testing.assert_array_equal(d, [0])
    ds.close()


def test_reordered_graph_rejected_in_batch(engine):
    g = gen.rmat(8, seed=3, weights=(1, 8))
    dg = engine.load(g, reorder=True)
    import torch
    o = torch.empty(g.n, dtype=torch.int32, device=engine.device)
    with pytest.raises(sx.SxError) as e:
        sx.sx_run_batch(engine.ctx, [(dg.handle, sx.SX_BFS, 0, o.data_ptr())], stream=engine.stream())
    assert e.value.status == sx.SX_EUNSUPPORTED
    dg.close()
