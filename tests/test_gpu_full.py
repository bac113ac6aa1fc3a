"""Parity at the full workload sizes, in the configuration bench.py times:
R-MAT scale 22 (BFS, SSSP, k-core), the 4096^2 grid (BFS, SSSP) and the
directed R-MAT scale 24 (PageRank within 1e-6 relative L1, k-core).  The
oracle computes every output element (serial C, seconds per run)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1812_04070_amd as sx
from paper_1812_04070_amd import gen
from tests.gpu_util import announce, rel_l1, run
from tests import pins

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def engine():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = sx.Engine(0)
    yield e
    e.close()


def test_rmat22(engine):
    g = gen.workload_graph("rmat22")
    src = gen.max_degree_vertex(g)
    dg = engine.load(g)
    announce("rmat22 bfs")
    d, st = run(engine, g, sx.SX_BFS, src, dg=dg)
    ref_d = oracle.bfs_g(g, src)
    np.testing.assert_array_equal(d, ref_d)
    announce("rmat22 sssp")
    x, st = run(engine, g, sx.SX_SSSP, src, dg=dg)
    np.testing.assert_array_equal(x, oracle.sssp_g(g, src))
    announce("rmat22 kcore")
    c, st = run(engine, g, sx.SX_KCORE, dg=dg)
    np.testing.assert_array_equal(c, oracle.kcore_g(g))
    # the forced arms give the same bytes at full size too
    for name, pol in [("push-only", sx.Policy(direction=sx.SX_DIR_PUSH)),
                      ("unfused", sx.Policy(fused=sx.SX_UNFUSED)),
                      ("fused", sx.Policy(fused=sx.SX_FUSED)),
                      ("fused-all", sx.Policy(fused=sx.SX_FUSED_ALL))]:
        announce(f"rmat22 bfs {name}")
        d2, _ = run(engine, g, sx.SX_BFS, src, pol, dg=dg)
        np.testing.assert_array_equal(d2, ref_d)
        if name.startswith("fused"):
            announce(f"rmat22 sssp {name}")
            x2, _ = run(engine, g, sx.SX_SSSP, src, pol, dg=dg)
            np.testing.assert_array_equal(x2, x)
    for k in (16, 32):
        announce(f"rmat22 kcore membership k={k}")
        out, _ = engine.run(dg, sx.SX_KCORE, -1, kcore_k=k)
        np.testing.assert_array_equal(engine.to_host(dg, sx.SX_KCORE, out), oracle.kcore_member_g(g, k))
        np.testing.assert_array_equal(engine.to_host(dg, sx.SX_KCORE, out), (c >= k).astype(np.int32))
    announce("rmat22 wcc")
    lab, _ = run(engine, g, sx.SX_WCC, -1, dg=dg)
    ref_w = oracle.wcc_g(g)
    np.testing.assert_array_equal(lab, ref_w)
    dg.close()
    # the degree-renumbered load that bench.py times
    dr = engine.load(g, reorder=True)
    announce("rmat22 reordered bfs / sssp / kcore")
    np.testing.assert_array_equal(run(engine, g, sx.SX_BFS, src, dg=dr)[0], ref_d)
    np.testing.assert_array_equal(run(engine, g, sx.SX_SSSP, src, dg=dr)[0], x)
    np.testing.assert_array_equal(run(engine, g, sx.SX_KCORE, dg=dr)[0], c)
    np.testing.assert_array_equal(run(engine, g, sx.SX_WCC, -1, dg=dr)[0], ref_w)
    dr.close()


def test_grid4096(engine):
    g = gen.workload_graph("grid4096")
    dg = engine.load(g)
    announce("grid4096 bfs")
    d, st = run(engine, g, sx.SX_BFS, 0, dg=dg)
    np.testing.assert_array_equal(d, oracle.bfs_g(g, 0))
    assert st["iterations"] >= 8000
    announce("grid4096 sssp")
    x, st = run(engine, g, sx.SX_SSSP, 0, dg=dg)
    ref = oracle.sssp_g(g, 0)
    np.testing.assert_array_equal(x, ref)
    announce("grid4096 sssp, automatic bucket width")
    x, st_auto = run(engine, g, sx.SX_SSSP, 0, dg=dg, sssp_delta=sx.SX_DELTA_AUTO)
    np.testing.assert_array_equal(x, ref)
    assert st_auto["edges_inspected"] < st["edges_inspected"] // 10
    announce("grid4096 bfs / sssp persistent (fused) arrangement")
    d2, st_f = run(engine, g, sx.SX_BFS, 0, sx.Policy(fused=sx.SX_FUSED), dg=dg)
    np.testing.assert_array_equal(d2, d)
    assert st_f["barrier_wait_ms"] > 0
    x2, _ = run(engine, g, sx.SX_SSSP, 0, sx.Policy(fused=sx.SX_FUSED), dg=dg)
    np.testing.assert_array_equal(x2, ref)
    announce("grid4096 wcc")
    lab, _ = run(engine, g, sx.SX_WCC, -1, dg=dg)
    np.testing.assert_array_equal(lab, oracle.wcc_g(g))
    dg.close()


def test_rmat24_directed(engine):
    g = gen.workload_graph("rmat24d")
    dg = engine.load(g)
    announce("rmat24d pagerank")
    r, st = run(engine, g, sx.SX_PAGERANK, dg=dg)
    ref = oracle.pagerank_g(g)
    err = rel_l1(r, ref)
    print(f"pagerank s24 rel L1 = {err:.3e}, {st['device_ms']:.2f} ms", flush=True)
    assert err <= 1e-6
    assert abs(float(r.astype(np.float64).sum()) - 1.0) < 1e-4
    announce("rmat24d kcore")
    c, st = run(engine, g, sx.SX_KCORE, dg=dg)
    ref_c = oracle.kcore_g(g)
    np.testing.assert_array_equal(c, ref_c)
    pins.kcore_certificate_fast(g.n, g.offsets, g.indices, c, g.in_offsets, g.in_indices)
    dg.close()
    dr = engine.load(g, reorder=True)
    announce("rmat24d reordered pagerank / kcore")
    r2, _ = run(engine, g, sx.SX_PAGERANK, dg=dr)
    assert rel_l1(r2, ref) <= 1e-6
    np.testing.assert_array_equal(run(engine, g, sx.SX_KCORE, dg=dr)[0], ref_c)
    dr.close()


def _trained_params():
    import json
    import os
    path = os.path.join(os.path.dirname(sx.__file__), "policy_mlp.json")
    with open(path) as f:
        return np.asarray(json.load(f)["params"], dtype=np.float32)


@pytest.mark.timeout(600)
def test_batch_workload_full(engine):
    """The batched workload at its full size (48 R-MAT graphs of scales 12-20,
    16 grids of sides 256-2048, 256 BFS/SSSP queries) in one launch, with the
    heuristic and with the trained policy: every query's output equals the
    oracle's."""
    import torch
    graphs, queries = gen.batch_workload()
    dgs = [engine.load(g) for g in graphs]
    algo = {"bfs": sx.SX_BFS, "sssp": sx.SX_SSSP}
    refs = [oracle.bfs_g(graphs[gi], s) if a == "bfs" else oracle.sssp_g(graphs[gi], s)
            for gi, a, s in queries]
    outs = [torch.empty(graphs[gi].n, dtype=torch.int32, device=engine.device) for gi, _, _ in queries]
    qs = [(dgs[gi].handle, algo[a], s, o.data_ptr()) for (gi, a, s), o in zip(queries, outs)]
    sx.sx_policy_load_mlp(engine.ctx, _trained_params())
    for pname, pol in [("heuristic", sx.Policy()), ("learned", sx.Policy(policy=sx.SX_POLICY_LEARNED))]:
        for o in outs:
            o.fill_(-7)
        announce(f"batch workload full {pname}")
        ms, _ = sx.sx_run_batch(engine.ctx, qs, pol.c(), sx.sx_batch_config(32, 0, 0), engine.stream())
        assert ms > 0
        for (gi, a, s), o, r in zip(queries, outs, refs):
            np.testing.assert_array_equal(engine.to_host(dgs[gi], algo[a], o), r)
    for d in dgs:
        d.close()
