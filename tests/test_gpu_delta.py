"""Parity of SSSP with delta-stepping buckets (Section 3.3): for every bucket
width the distances must equal the oracle's Dijkstra bit for bit, in every
arrangement (the persistent and unfused ones relax without buckets), with
the JIT, online and ballot filters, and when a run switches to pull steps."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1812_04070_amd as sx
from paper_1812_04070_amd import gen
from tests.gpu_util import announce, run

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
    ("grid-61", lambda: gen.grid(61, 0.1, seed=7, weights=(1, 1000))),
    ("grid-40-unit", lambda: gen.grid(40, 0.0, seed=3, weights=(1, 1))),
    ("rmat12", lambda: gen.rmat(12, seed=6, weights=(1, 64))),
    ("rmat15", lambda: gen.rmat(15, seed=16, weights=(1, 64))),
    ("er-130-dense", lambda: gen.random_graph(130, 0.3, seed=2, weights=(1, 9))),
    # a path whose weights fall along it: every vertex lands in its own bucket
    ("path-300-falling", lambda: gen.from_edges(300, [(i, i + 1) for i in range(299)],
                                                 [1000 - 3 * i for i in range(299)])),
    ("star-3000", lambda: gen.from_edges(3001, [(0, i) for i in range(1, 3001)], list(range(1, 3001)))),
    ("matching-plus-isolated", lambda: gen.from_edges(500, [(2 * i, 2 * i + 1) for i in range(200)],
                                                       [1 + i % 7 for i in range(200)])),
]

DELTAS = [1, 7, 64, 1000, sx.SX_DELTA_AUTO, 1 << 31]

POLICIES = [
    ("auto", sx.Policy()),
    ("seq-online", sx.Policy(filter=sx.SX_FILTER_ONLINE, fused=sx.SX_SEQUENCED)),
    ("seq-ballot", sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_BALLOT, fused=sx.SX_SEQUENCED)),
    ("seq-tiny-bins", sx.Policy(bin_small=4, bin_large=8, online_cap=1)),
    ("pull", sx.Policy(direction=sx.SX_DIR_PULL)),
    ("fused", sx.Policy(fused=sx.SX_FUSED)),
    ("unfused", sx.Policy(fused=sx.SX_UNFUSED)),
]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_delta_stepping_exact(engine, name, make):
    g = make()
    srcs = [gen.max_degree_vertex(g), int(np.flatnonzero(g.out_degree())[-1])]
    dg = engine.load(g)
    for s in srcs:
        ref = oracle.sssp_g(g, s)
        base_edges = None
        for delta in DELTAS:
            for pname, pol in POLICIES:
                announce(f"delta {name} src={s} delta={delta} {pname}")
                x, st = run(engine, g, sx.SX_SSSP, s, pol, dg=dg, sssp_delta=delta)
                np.testing.assert_array_equal(x, ref)
                if pname == "auto" and delta == DELTAS[-1]:
                    base_edges = st["edges_inspected"]
    dg.close()
    assert base_edges is not None


def test_delta_cuts_relaxations_on_grid(engine):
    """On a grid with weights spread over [1, 1000] the buckets remove most
    re-expansions (a property of the schedule, checked loosely)."""
    g = gen.grid(128, 0.1, seed=11, weights=(1, 1000))
    s = gen.max_degree_vertex(g)
    ref = oracle.sssp_g(g, s)
    dg = engine.load(g)
    announce("delta grid-128 without buckets")
    x0, st0 = run(engine, g, sx.SX_SSSP, s, None, dg=dg)
    announce("delta grid-128 delta=500")
    x1, st1 = run(engine, g, sx.SX_SSSP, s, None, dg=dg, sssp_delta=500)
    announce("delta grid-128 automatic width (a graph this small stays unbucketed)")
    x2, st2 = run(engine, g, sx.SX_SSSP, s, None, dg=dg, sssp_delta=sx.SX_DELTA_AUTO)
    dg.close()
    np.testing.assert_array_equal(x0, ref)
    np.testing.assert_array_equal(x1, ref)
    np.testing.assert_array_equal(x2, ref)
    print(f"[delta] grid-128 arcs inspected: none {st0['edges_inspected']} delta=500 {st1['edges_inspected']}; "
          f"iterations {st0['iterations']} -> {st1['iterations']}")
    assert st1["edges_inspected"] < st0["edges_inspected"]
    assert st2["iterations"] == st0["iterations"]


def test_delta_auto_keeps_dense_graphs_unbucketed(engine):
    """The automatic width leaves graphs of 8+ arcs per vertex without
    buckets: the same iterations as the plain run (the full-size grid test
    checks that it does bucket the 4096^2 grid)."""
    g = gen.rmat(14, seed=5, weights=(1, 64))
    assert g.m >= 8 * g.n
    s = gen.max_degree_vertex(g)
    dg = engine.load(g)
    announce("delta rmat14 none / auto")
    x0, st0 = run(engine, g, sx.SX_SSSP, s, None, dg=dg)
    x1, st1 = run(engine, g, sx.SX_SSSP, s, None, dg=dg, sssp_delta=sx.SX_DELTA_AUTO)
    dg.close()
    np.testing.assert_array_equal(x0, oracle.sssp_g(g, s))
    np.testing.assert_array_equal(x1, x0)
    assert st1["iterations"] == st0["iterations"]


def test_delta_single_and_edgeless(engine):
    one = gen.from_edges(1, [], [])
    announce("delta single vertex")
    x, _ = run(engine, one, sx.SX_SSSP, 0, None, sssp_delta=5)
    np.testing.assert_array_equal(x, [0])
    two = gen.from_edges(2, [], [])
    announce("delta two isolated vertices")
    x, _ = run(engine, two, sx.SX_SSSP, 1, None, sssp_delta=5)
    np.testing.assert_array_equal(x, [0xFFFFFFFF, 0])


def test_delta_same_as_plain_on_reordered_rmat(engine):
    g = gen.rmat(16, seed=21, weights=(1, 64))
    s = gen.max_degree_vertex(g)
    ref = oracle.sssp_g(g, s)
    dg = engine.load(g, reorder=True)
    for delta in (16, 64, 256):
        announce(f"delta reordered rmat16 delta={delta}")
        x, _ = run(engine, g, sx.SX_SSSP, s, None, dg=dg, sssp_delta=delta)
        np.testing.assert_array_equal(x, ref)
    dg.close()


def test_delta_auto_engages_late(engine):
    """On a grid of 2^21+ vertices the automatic width engages after the
    first 64 iterations, from the bucket of the smallest listed distance;
    exact under every filter, and far fewer arcs than without buckets."""
    g = gen.grid(1500, 0.1, seed=13, weights=(1, 1000))
    assert g.n >= 1 << 21 and g.m < 8 * g.n
    s = gen.max_degree_vertex(g)
    ref = oracle.sssp_g(g, s)
    dg = engine.load(g)
    announce("delta grid-1500 without buckets")
    x0, st0 = run(engine, g, sx.SX_SSSP, s, None, dg=dg)
    np.testing.assert_array_equal(x0, ref)
    for pname, pol in POLICIES[:4]:
        announce(f"delta grid-1500 automatic width {pname}")
        x, st = run(engine, g, sx.SX_SSSP, s, pol, dg=dg, sssp_delta=sx.SX_DELTA_AUTO)
        np.testing.assert_array_equal(x, ref)
        assert st["edges_inspected"] < st0["edges_inspected"] // 4, pname
    dg.close()
