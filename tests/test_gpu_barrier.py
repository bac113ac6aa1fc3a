"""The software global barrier's watchdog and its stall statistics.

The watchdog is forced from the host with a tiny wait budget (1 us of wall
clock): at the first barrier of a persistent run every early workgroup waits
for the one processing the hub source far longer than that, so the run
must end with SX_EDEADLOCK -- every wait is bounded, so every workgroup
leaves the kernel normally -- and the next run on the same graph must be
exact again.  barrier_wait_ms is checked for sanity in each arrangement."""
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


@pytest.mark.parametrize("algo", [sx.SX_BFS, sx.SX_SSSP, sx.SX_KCORE, sx.SX_PAGERANK])
def test_watchdog_fires_and_run_recovers(engine, algo):
    g = gen.rmat(14, seed=2, weights=(1, 64))
    src = gen.max_degree_vertex(g) if algo in (sx.SX_BFS, sx.SX_SSSP) else -1
    dg = engine.load(g)
    announce(f"watchdog algo={algo}: 1 us budget")
    tiny = sx.Policy(fused=sx.SX_FUSED, watchdog_us=1)
    with pytest.raises(sx.SxError) as ei:
        engine.run(dg, algo, src, tiny)
    assert ei.value.status == sx.SX_EDEADLOCK
    announce(f"watchdog algo={algo}: recovery run")
    h, st = run(engine, g, algo, src, sx.Policy(fused=sx.SX_FUSED), dg=dg)
    ref = {sx.SX_BFS: lambda: oracle.bfs_g(g, src), sx.SX_SSSP: lambda: oracle.sssp_g(g, src),
           sx.SX_KCORE: lambda: oracle.kcore_g(g), sx.SX_PAGERANK: None}[algo]
    if ref is not None:
        np.testing.assert_array_equal(h, ref())
    else:
        r = oracle.pagerank_g(g)
        assert np.abs(h - r).sum() / np.abs(r).sum() <= 1e-6
    dg.close()


def test_watchdog_negative_rejected(engine):
    p = engine.program(sx.SX_BFS)
    with pytest.raises(sx.SxError):
        sx.sx_program_set_policy(p, sx.Policy(watchdog_us=-1).c())


@pytest.mark.parametrize("fused", [sx.SX_SEQUENCED, sx.SX_FUSED, sx.SX_FUSED_ALL, sx.SX_UNFUSED])
def test_barrier_wait_reported(engine, fused):
    g = gen.rmat(15, seed=5, weights=(1, 64))
    src = gen.max_degree_vertex(g)
    dg = engine.load(g)
    for algo in (sx.SX_BFS, sx.SX_SSSP, sx.SX_KCORE):
        if algo == sx.SX_KCORE and fused == sx.SX_FUSED_ALL:
            continue
        announce(f"barrier wait algo={algo} fused={fused}")
        # (k-core on the grid: on a graph this small the one-workgroup tail
        # would take the whole decomposition, with no grid barrier)
        _, st = run(engine, g, algo, src if algo != sx.SX_KCORE else -1,
                    sx.Policy(fused=fused, kcore_tail=-1), dg=dg)
        w = st["barrier_wait_ms"]
        if fused == sx.SX_UNFUSED and algo != sx.SX_KCORE:
            assert w == 0.0
        else:
            assert 0.0 < w <= st["device_ms"] * 1.05, (w, st["device_ms"])
    dg.close()
