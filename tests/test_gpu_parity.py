"""Parity of the HIP engine (through the C ABI) with the CPU oracle.

BFS, SSSP and k-core are compared element by element and must be identical;
PageRank (FP32) must be within 1e-6 relative L1 of the FP64 oracle.  Every
policy arm (direction, filter, bins, fusion, grid size) must give the same
integer output: the method's choices change the schedule, never the result.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import oracle
import paper_1812_04070_amd as sx
from paper_1812_04070_amd import gen
from tests.gpu_util import ARMS, announce, rel_l1, run

pytestmark = pytest.mark.gpu

PR_TOL = 1e-6


@pytest.fixture(scope="module")
def engine():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = sx.Engine(0)
    yield e
    e.close()


def _example():
    edges = [(0, 1), (0, 3), (3, 2), (3, 4), (2, 1), (2, 5), (4, 5), (4, 6), (4, 7), (4, 8)]
    w = [5, 1, 1, 2, 2, 3, 1, 2, 3, 4]
    return gen.from_edges(9, edges, w, name="worked-example")


SMALL_GRAPHS = [
    ("worked-example", _example),
    ("er-70", lambda: gen.random_graph(70, 0.08, seed=1, weights=(1, 64))),
    ("er-130-dense", lambda: gen.random_graph(130, 0.3, seed=2, weights=(1, 9))),
    ("rmat10", lambda: gen.rmat(10, seed=5, weights=(1, 64))),
    ("rmat12", lambda: gen.rmat(12, seed=6, weights=(1, 64))),
    ("grid-37", lambda: gen.grid(37, 0.1, seed=7, weights=(1, 1000))),
    ("path-1000", lambda: gen.from_edges(1000, [(i, i + 1) for i in range(999)], [3] * 999)),
    ("star-3000", lambda: gen.from_edges(3001, [(0, i) for i in range(1, 3001)], list(range(1, 3001)))),
]


@pytest.mark.parametrize("name,make", SMALL_GRAPHS, ids=[s[0] for s in SMALL_GRAPHS])
@pytest.mark.parametrize("arm", ARMS, ids=[a[0] for a in ARMS])
def test_bfs_sssp_small(engine, name, make, arm):
    g = make()
    src = gen.max_degree_vertex(g)
    dg = engine.load(g)
    announce(f"bfs {name} {arm[0]} src={src}")
    d, st = run(engine, g, sx.SX_BFS, src, arm[1], dg=dg)
    np.testing.assert_array_equal(d, oracle.bfs_g(g, src))
    announce(f"sssp {name} {arm[0]} src={src}")
    x, st = run(engine, g, sx.SX_SSSP, src, arm[1], dg=dg)
    np.testing.assert_array_equal(x, oracle.sssp_g(g, src))
    dg.close()


@pytest.mark.parametrize("name,make", SMALL_GRAPHS, ids=[s[0] for s in SMALL_GRAPHS])
def test_kcore_small(engine, name, make):
    """Graphs this small go to the one-workgroup tail at once (kcore_tail
    default); with kcore_tail = -1 every arm peels on the grid."""
    g = make()
    ref = oracle.kcore_g(g)
    for arm in ARMS:
        for tail in (0, -1):
            announce(f"kcore {name} {arm[0]} tail={tail}")
            c, _ = run(engine, g, sx.SX_KCORE, -1, dataclasses.replace(arm[1], kcore_tail=tail))
            np.testing.assert_array_equal(c, ref)


def test_sources_and_isolated(engine):
    g = gen.rmat(11, seed=3, weights=(1, 64))
    dg = engine.load(g)
    deg = g.out_degree()
    iso = int(np.nonzero(deg == 0)[0][0])
    for s in [0, iso, g.n - 1, int(np.argmin(np.where(deg > 0, deg, 10**9)))]:
        announce(f"bfs/sssp rmat11 src={s}")
        d, _ = run(engine, g, sx.SX_BFS, s, dg=dg)
        np.testing.assert_array_equal(d, oracle.bfs_g(g, s))
        x, _ = run(engine, g, sx.SX_SSSP, s, dg=dg)
        np.testing.assert_array_equal(x, oracle.sssp_g(g, s))
    dg.close()


def test_degenerate_graphs(engine):
    one = gen.from_edges(1, [], [])
    one.weights = np.zeros(0, dtype=np.uint32)
    announce("single vertex")
    d, _ = run(engine, one, sx.SX_BFS, 0)
    assert d.tolist() == [0]
    x, _ = run(engine, one, sx.SX_SSSP, 0)
    assert x.tolist() == [0]
    c, _ = run(engine, one, sx.SX_KCORE)
    assert c.tolist() == [0]
    edgeless = gen.from_edges(100, [], directed=True)
    announce("edgeless pagerank")
    r, _ = run(engine, edgeless, sx.SX_PAGERANK)
    np.testing.assert_allclose(r, np.full(100, 0.01), rtol=1e-6)


def test_invalid_arguments(engine):
    g = gen.rmat(8, seed=1, weights=(1, 4))
    dg = engine.load(g)
    with pytest.raises(sx.SxError) as e:
        engine.run(dg, sx.SX_BFS, g.n)
    assert e.value.status == sx.SX_EINVAL
    with pytest.raises(sx.SxError) as e:
        engine.run(dg, sx.SX_BFS, -1)
    assert e.value.status == sx.SX_EINVAL
    gu = gen.rmat(8, seed=1)
    dgu = engine.load(gu)
    with pytest.raises(sx.SxError) as e:
        engine.run(dgu, sx.SX_SSSP, 0)
    assert e.value.status == sx.SX_EINVAL
    with pytest.raises(sx.SxError):
        engine.run(dg, sx.SX_BFS, 0, sx.Policy(direction=7))
    dg.close()
    dgu.close()


@pytest.mark.parametrize("scale", [10, 14])
def test_pagerank_directed(engine, scale):
    g = gen.rmat(scale, seed=4, directed=True)
    announce(f"pagerank rmat{scale}d")
    r, st = run(engine, g, sx.SX_PAGERANK)
    ref = oracle.pagerank_g(g)
    err = rel_l1(r, ref)
    assert err <= PR_TOL, err
    # deterministic: bitwise identical on a second run
    r2, _ = run(engine, g, sx.SX_PAGERANK)
    assert np.array_equal(r.view(np.uint32), r2.view(np.uint32))


def test_pagerank_undirected_and_iters(engine):
    g = gen.rmat(12, seed=8)
    for iters in [1, 3, 20]:
        announce(f"pagerank rmat12u iters={iters}")
        r, _ = run(engine, g, sx.SX_PAGERANK, pr_iters=iters)
        assert rel_l1(r, oracle.pagerank_g(g, 0.85, iters)) <= PR_TOL


def test_kcore_directed(engine):
    g = gen.rmat(13, seed=4, directed=True)
    announce("kcore rmat13d")
    c, _ = run(engine, g, sx.SX_KCORE)
    np.testing.assert_array_equal(c, oracle.kcore_g(g))


def test_rmat16_workload(engine):
    """The s16 workload: BFS over every arm, SSSP and k-core."""
    g = gen.workload_graph("rmat16")
    src = gen.max_degree_vertex(g)
    dg = engine.load(g)
    ref_d = oracle.bfs_g(g, src)
    ref_x = oracle.sssp_g(g, src)
    for name, pol in ARMS:
        announce(f"rmat16 bfs {name}")
        d, st = run(engine, g, sx.SX_BFS, src, pol, dg=dg)
        np.testing.assert_array_equal(d, ref_d)
        announce(f"rmat16 sssp {name}")
        x, st = run(engine, g, sx.SX_SSSP, src, pol, dg=dg)
        np.testing.assert_array_equal(x, ref_x)
    announce("rmat16 kcore")
    c, _ = run(engine, g, sx.SX_KCORE, dg=dg)
    np.testing.assert_array_equal(c, oracle.kcore_g(g))
    dg.close()


@pytest.mark.parametrize("scale", [18, 20])
def test_kcore_pull_steps(engine, scale):
    """Dense last levels of R-MAT s18 / s20 take pull steps whose large
    candidates are split into chunks settled by different workgroups (one of
    them may delete the vertex while another reads it).  Every direction and
    both kernel arrangements must give the oracle's core numbers."""
    g = gen.rmat(scale, seed=2)
    ref = oracle.kcore_g(g)
    dg = engine.load(g)
    # the grid peels every level (no one-workgroup tail), where the pull
    # steps of the dense last levels are
    for name, pol in [("auto", sx.Policy(kcore_tail=-1)), ("auto-fused", sx.Policy(fused=sx.SX_FUSED)),
                      ("pull", sx.Policy(direction=sx.SX_DIR_PULL, kcore_tail=-1)),
                      ("push-fused", sx.Policy(fused=sx.SX_FUSED, direction=sx.SX_DIR_PUSH)),
                      ("ballot", sx.Policy(filter=sx.SX_FILTER_BALLOT, kcore_tail=-1))]:
        announce(f"kcore rmat{scale} {name}")
        c, st = run(engine, g, sx.SX_KCORE, -1, pol, dg=dg)
        np.testing.assert_array_equal(c, ref)
        if name == "auto":
            assert st["pull_iters"] > 0
    dg.close()


def test_kcore_directed_pull(engine):
    g = gen.rmat(16, seed=4, directed=True)
    ref = oracle.kcore_g(g)
    for name, pol in [("auto", sx.Policy()), ("auto-grid", sx.Policy(kcore_tail=-1)),
                      ("pull", sx.Policy(direction=sx.SX_DIR_PULL, kcore_tail=-1)),
                      ("fused", sx.Policy(fused=sx.SX_FUSED))]:
        announce(f"kcore rmat16d {name}")
        c, _ = run(engine, g, sx.SX_KCORE, -1, pol)
        np.testing.assert_array_equal(c, ref)


def test_expansion_record_long_lists(engine):
    """Steps whose lists hold 2^16 vertices or more skip a listed vertex whose
    distance (label) equals the one its last expansion started from.  R-MAT
    s18 reaches such lists: SSSP in every arrangement and from two sources
    in a row on one loaded graph (the second run must not meet the first
    run's record), a directed SSSP, and WCC; all identical to the oracle."""
    g = gen.rmat(18, seed=21, weights=(1, 64))
    dg = engine.load(g)
    deg = np.diff(g.offsets)
    srcs = [gen.max_degree_vertex(g), int(np.nonzero(deg == 1)[0][0])]
    pols = [("auto", sx.Policy()), ("push-only", sx.Policy(direction=sx.SX_DIR_PUSH)),
            ("ballot", sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_BALLOT)),
            ("fused", sx.Policy(fused=sx.SX_FUSED)), ("fused-all", sx.Policy(fused=sx.SX_FUSED_ALL)),
            ("unfused", sx.Policy(fused=sx.SX_UNFUSED))]
    long_list = False
    for src in srcs:
        ref = oracle.sssp_g(g, src)
        for name, pol in pols:
            announce(f"expansion record sssp src={src} {name}")
            x, st = run(engine, g, sx.SX_SSSP, src, pol, dg=dg)
            np.testing.assert_array_equal(x, ref)
            long_list = long_list or st["vertex_expansions"] >= (1 << 16)
    assert long_list
    ref_w = oracle.wcc_g(g)
    for name, pol in pols:
        announce(f"expansion record wcc {name}")
        np.testing.assert_array_equal(run(engine, g, sx.SX_WCC, -1, pol, dg=dg)[0], ref_w)
    dg.close()
    gd = gen.rmat(18, seed=22, weights=(1, 64), directed=True)
    src = gen.max_degree_vertex(gd)
    announce("expansion record directed sssp")
    np.testing.assert_array_equal(run(engine, gd, sx.SX_SSSP, src)[0], oracle.sssp_g(gd, src))


@pytest.mark.parametrize("case", ["rmat16", "rmat18", "rmat16d", "grid-150", "er-20000"])
def test_kcore_tail(engine, case):
    """The one-workgroup tail of the decomposition: taken over at several
    sizes (from the first level on for the default on small graphs, at a
    few hundred or thousand vertices, never), on undirected and directed
    R-MAT, a grid and a sparse random graph; every result equal to the
    oracle's."""
    g = {"rmat16": lambda: gen.rmat(16, seed=31), "rmat18": lambda: gen.rmat(18, seed=32),
         "rmat16d": lambda: gen.rmat(16, seed=33, directed=True),
         "grid-150": lambda: gen.grid(150, 0.1, seed=34),
         "er-20000": lambda: gen.random_graph(20000, 0.0008, seed=35)}[case]()
    ref = oracle.kcore_g(g)
    dg = engine.load(g)
    for tail in (0, 4096, 300, 1, -1):
        announce(f"kcore tail {case} kcore_tail={tail}")
        c, st = run(engine, g, sx.SX_KCORE, -1, sx.Policy(kcore_tail=tail), dg=dg)
        np.testing.assert_array_equal(c, ref)
    dg.close()


def test_kcore_multigraph(engine):
    """Parallel arcs count once each in a degree (the oracle's definition
    too): every arc of R-MAT s12 doubled.  The one-workgroup tail sizes its
    rows by the current degree, parallel arcs included, and must agree with
    the grid and the oracle."""
    import dataclasses as dc
    g = gen.rmat(12, seed=41)
    deg = np.diff(g.offsets)
    off2 = (2 * g.offsets).astype(np.int32)
    idx2 = np.repeat(g.indices, 2).astype(np.int32)
    mg = dc.replace(g, offsets=off2, indices=idx2, name="rmat12-doubled")
    assert mg.m == 2 * g.m and np.array_equal(np.diff(mg.offsets), 2 * deg)
    ref = oracle.kcore_g(mg)
    assert np.array_equal(ref, 2 * oracle.kcore_g(g))   # doubling every arc doubles every core
    for tail in (0, 2000, -1):
        announce(f"kcore multigraph kcore_tail={tail}")
        c, _ = run(engine, mg, sx.SX_KCORE, -1, sx.Policy(kcore_tail=tail))
        np.testing.assert_array_equal(c, ref)


@pytest.mark.skip(reason="level scans that peel their own finds were removed: the build that carried "
                         "them gave wrong core numbers (one level low) on the plain ballot arm of R-MAT "
                         "s20, which does not take that path, and one run did not end; the cause was not "
                         "found, and the policy field kcore_scan_peel this test sets no longer exists")
@pytest.mark.parametrize("case", ["rmat16", "rmat18", "rmat16d", "grid-150", "er-20000", "star-3000",
                                  "rmat12-doubled"])
def test_kcore_scan_peel(engine, case):
    """Level scans that delete their own finds in the same launch (the
    default) against scans that only list them: the grid peels every level
    (no tail), with the default bins, push only, a one-entry online list (the
    next step's list overflows and a plain scan recovers it), eight
    workgroups (finds overflow a workgroup's queue and arc budget), and the
    fixed-k membership; every result equal to the oracle's."""
    import dataclasses as dc
    if case == "rmat12-doubled":
        g0 = gen.rmat(12, seed=41)
        g = dc.replace(g0, offsets=(2 * g0.offsets).astype(np.int32),
                       indices=np.repeat(g0.indices, 2).astype(np.int32), name=case)
    else:
        g = {"rmat16": lambda: gen.rmat(16, seed=51), "rmat18": lambda: gen.rmat(18, seed=52),
             "rmat16d": lambda: gen.rmat(16, seed=53, directed=True),
             "grid-150": lambda: gen.grid(150, 0.1, seed=54),
             "er-20000": lambda: gen.random_graph(20000, 0.0008, seed=55),
             "star-3000": lambda: gen.from_edges(3001, [(0, i) for i in range(1, 3001)])}[case]()
    ref = oracle.kcore_g(g)
    dg = engine.load(g)
    try:
        _scan_peel_arms(engine, g, dg, ref, case)
    finally:
        dg.close()


def _scan_peel_arms(engine, g, dg, ref, case):
    import dataclasses as dc
    launches = {}
    for sp in (0, -1):
        for name, pol in [("auto", sx.Policy()), ("push", sx.Policy(direction=sx.SX_DIR_PUSH)),
                          ("tiny-online", sx.Policy(bin_small=4, bin_large=8, online_cap=1)),
                          ("grid-8", sx.Policy(grid_wgs=8))]:
            pol = dc.replace(pol, kcore_tail=-1, kcore_scan_peel=sp)
            announce(f"kcore scan-peel {case} {name} scan_peel={sp}")
            c, st = run(engine, g, sx.SX_KCORE, -1, pol, dg=dg)
            np.testing.assert_array_equal(c, ref)
            launches[(name, sp)] = st["launches"]
        for k in (2, int(ref.max())):
            announce(f"kcore scan-peel {case} member k={k} scan_peel={sp}")
            out, _ = engine.run(dg, sx.SX_KCORE, -1, sx.Policy(kcore_scan_peel=sp), kcore_k=k)
            np.testing.assert_array_equal(engine.to_host(dg, sx.SX_KCORE, out), oracle.kcore_member_g(g, k))
    print(f"[scan-peel] {case} launches (on, off): "
          + ", ".join(f"{n} {launches[(n, 0)]}/{launches[(n, -1)]}" for n in ("auto", "push", "tiny-online", "grid-8")),
          flush=True)
