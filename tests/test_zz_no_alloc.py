"""sx_run_static, the entry point that allocates nothing (its workspace is the
library's static device array), against sx_run on the same graph: identical
outputs for BFS, SSSP and WCC on two calls in a row, the second on a smaller
graph (the array keeps the first call's contents), in the sequenced and
persistent arrangements; an oversize graph and the unsupported cases are
rejected before any kernel runs."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1812_04070_amd as sx
from paper_1812_04070_amd import gen
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def engine():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = sx.Engine(0)
    yield e
    e.close()


POLICIES = [("sequenced", sx.Policy()), ("fused", sx.Policy(fused=sx.SX_FUSED)),
            ("fused-all-pull", sx.Policy(fused=sx.SX_FUSED_ALL, direction=sx.SX_DIR_PULL))]


@pytest.mark.parametrize("pname,pol", POLICIES, ids=[p[0] for p in POLICIES])
def test_static_matches_run_two_calls(engine, pname, pol):
    big = gen.rmat(15, seed=11, weights=(1, 64))
    small = gen.grid(40, 0.2, seed=5, weights=(1, 50))
    for gi, g in enumerate((big, small)):
        dg = engine.load(g)
        src = gen.max_degree_vertex(g)
        for algo, s in ((sx.SX_BFS, src), (sx.SX_SSSP, src), (sx.SX_WCC, -1)):
            announce(f"static {pname} graph={gi} n={g.n} algo={algo}")
            o1, st1 = engine.run_static(dg, algo, s, pol)
            h1 = engine.to_host(dg, algo, o1)
            o2, st2 = engine.run(dg, algo, s, pol)
            h2 = engine.to_host(dg, algo, o2)
            np.testing.assert_array_equal(h1, h2)
            ref = {sx.SX_BFS: lambda: oracle.bfs_g(g, s), sx.SX_SSSP: lambda: oracle.sssp_g(g, s),
                   sx.SX_WCC: lambda: oracle.wcc_g(g)}[algo]()
            np.testing.assert_array_equal(h1, ref)
            if algo == sx.SX_BFS:
                # BFS levels are fixed by the graph; the work of the minimum
                # programs depends on the order of their atomic updates
                assert st1["iterations"] == st2["iterations"]
        dg.close()


def test_static_rejects(engine):
    g = gen.rmat(10, seed=3, weights=(1, 64))
    dg = engine.load(g)
    p = engine.program(sx.SX_BFS)
    import torch
    out = torch.empty(g.n, dtype=torch.int32, device=engine.device)
    # a graph whose workspace exceeds the static array: rejected from its
    # sizes alone (the borrowed arrays are never read)
    huge = sx.sx_graph_desc(1 << 26, dg.desc.m, dg.desc.offsets, dg.desc.indices, dg.desc.weights,
                            None, None, None, dg.desc.flags)
    sx.sx_program_set_policy(p, sx.Policy().c())
    announce("static oversize")
    with pytest.raises(sx.SxError) as ei:
        sx.sx_run_static(p, huge, 0, out.data_ptr(), engine.stream())
    assert ei.value.status == sx.SX_EINVAL and "static workspace" in str(ei.value)
    announce("static unfused / kcore / no device pointers")
    sx.sx_program_set_policy(p, sx.Policy(fused=sx.SX_UNFUSED).c())
    with pytest.raises(sx.SxError) as ei:
        sx.sx_run_static(p, dg.desc, 0, out.data_ptr(), engine.stream())
    assert ei.value.status == sx.SX_EUNSUPPORTED
    pk = engine.program(sx.SX_KCORE)
    with pytest.raises(sx.SxError) as ei:
        sx.sx_run_static(pk, dg.desc, -1, out.data_ptr(), engine.stream())
    assert ei.value.status == sx.SX_EUNSUPPORTED
    host = sx.sx_graph_desc(dg.desc.n, dg.desc.m, dg.desc.offsets, dg.desc.indices, dg.desc.weights,
                            None, None, None, sx.SX_UNDIRECTED)
    sx.sx_program_set_policy(p, sx.Policy().c())
    with pytest.raises(sx.SxError) as ei:
        sx.sx_run_static(p, host, 0, out.data_ptr(), engine.stream())
    assert ei.value.status == sx.SX_EINVAL
    # the engine still runs normally afterwards
    announce("static after rejections")
    o, _ = engine.run_static(dg, sx.SX_BFS, 0)
    np.testing.assert_array_equal(engine.to_host(dg, sx.SX_BFS, o), oracle.bfs_g(g, 0))
    dg.close()
