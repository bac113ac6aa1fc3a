"""Parity of connected components (minimum-label propagation, SX_WCC) and of
the paper's fixed-k k-core membership (SX_KCORE with kcore_k > 0) with the
oracle, under every arrangement and forced direction / filter; edge cases
(isolated vertices, a single vertex, no arcs, k above every degree)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1812_04070_amd as sx
from paper_1812_04070_amd import gen
from tests.gpu_util import ARMS, announce, run

pytestmark = pytest.mark.gpu

WCC_ARMS = ARMS + [
    ("push-fused-all", sx.Policy(direction=sx.SX_DIR_PUSH, fused=sx.SX_FUSED_ALL)),
    ("auto-fused-all", sx.Policy(fused=sx.SX_FUSED_ALL)),
    ("push-online-seq", sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_ONLINE, fused=sx.SX_SEQUENCED)),
    ("push-jit-unfused", sx.Policy(direction=sx.SX_DIR_PUSH, fused=sx.SX_UNFUSED)),
]


@pytest.fixture(scope="module")
def engine():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = sx.Engine(0)
    yield e
    e.close()


def _two_paths():
    return gen.from_edges(9, [(8, 6), (6, 4), (4, 2), (7, 5), (5, 3), (3, 1)])


WCC_GRAPHS = [
    ("two-paths", _two_paths),
    ("er-300-sparse", lambda: gen.random_graph(300, 0.004, seed=3)),
    ("rmat12", lambda: gen.rmat(12, seed=6)),
    ("rmat14", lambda: gen.rmat(14, seed=9)),
    ("grid-70-holes", lambda: gen.grid(70, 0.45, seed=7)),
    ("path-2000-reversed", lambda: gen.from_edges(2000, [(i, i + 1) for i in range(1999)])),
    ("star-3000", lambda: gen.from_edges(3001, [(0, i) for i in range(1, 3001)])),
    ("edgeless-100", lambda: gen.from_edges(100, [])),
]


@pytest.mark.parametrize("name,make", WCC_GRAPHS, ids=[s[0] for s in WCC_GRAPHS])
@pytest.mark.parametrize("arm", WCC_ARMS, ids=[a[0] for a in WCC_ARMS])
def test_wcc_small(engine, name, make, arm):
    g = make()
    ref = oracle.wcc_g(g)
    announce(f"wcc {name} {arm[0]}")
    lab, st = run(engine, g, sx.SX_WCC, -1, arm[1])
    np.testing.assert_array_equal(lab, ref)


def test_wcc_single_vertex_and_directed(engine):
    g1 = gen.from_edges(1, [])
    announce("wcc single vertex")
    lab, _ = run(engine, g1, sx.SX_WCC, -1)
    assert lab.tolist() == [0]
    gd = gen.random_graph(50, 0.05, seed=1, directed=True)
    dg = engine.load(gd)
    announce("wcc directed -> unsupported")
    with pytest.raises(sx.SxError) as ei:
        engine.run(dg, sx.SX_WCC, -1)
    assert ei.value.status == sx.SX_EUNSUPPORTED
    dg.close()


KC_GRAPHS = [
    ("er-130-dense", lambda: gen.random_graph(130, 0.3, seed=2)),
    ("rmat12", lambda: gen.rmat(12, seed=6)),
    ("rmat13-directed", lambda: gen.rmat(13, seed=4, directed=True)),
    ("grid-50", lambda: gen.grid(50, 0.1, seed=7)),
    ("clique-40-plus-path", lambda: gen.from_edges(
        60, [(i, j) for i in range(40) for j in range(i + 1, 40)] + [(i, i + 1) for i in range(39, 59)])),
]
KC_ARMS = [("auto", sx.Policy()),
           ("push-seq", sx.Policy(direction=sx.SX_DIR_PUSH)),
           ("pull-seq", sx.Policy(direction=sx.SX_DIR_PULL)),
           ("ballot-seq", sx.Policy(filter=sx.SX_FILTER_BALLOT)),
           ("tiny-bins-jit", sx.Policy(bin_small=4, bin_large=8, online_cap=1)),
           ("fused", sx.Policy(fused=sx.SX_FUSED)),
           ("fused-pull", sx.Policy(fused=sx.SX_FUSED, direction=sx.SX_DIR_PULL))]


@pytest.mark.parametrize("name,make", KC_GRAPHS, ids=[s[0] for s in KC_GRAPHS])
@pytest.mark.parametrize("arm", KC_ARMS, ids=[a[0] for a in KC_ARMS])
def test_kcore_membership_small(engine, name, make, arm):
    g = make()
    core = oracle.kcore_g(g)
    dg = engine.load(g)
    for k in (1, 2, 3, 5, 16, 32, int(core.max()), int(core.max()) + 1):
        announce(f"kcore member {name} {arm[0]} k={k}")
        out, st = engine.run(dg, sx.SX_KCORE, -1, arm[1], kcore_k=k)
        got = engine.to_host(dg, sx.SX_KCORE, out)
        np.testing.assert_array_equal(got, oracle.kcore_member_g(g, k))
        assert np.array_equal(got, (core >= k).astype(np.int32))
    dg.close()


def test_kcore_membership_reordered(engine):
    g = gen.rmat(14, seed=3)
    dg = engine.load(g, reorder=True)
    for k in (4, 16, 32):
        announce(f"kcore member reordered k={k}")
        out, _ = engine.run(dg, sx.SX_KCORE, -1, kcore_k=k)
        np.testing.assert_array_equal(engine.to_host(dg, sx.SX_KCORE, out), oracle.kcore_member_g(g, k))
    dg.close()


def test_kcore_k_negative_rejected(engine):
    with pytest.raises(sx.SxError) as ei:
        sx.sx_program_register(engine.ctx, sx.SX_KCORE, kcore_k=-1)
    assert ei.value.status == sx.SX_EINVAL
