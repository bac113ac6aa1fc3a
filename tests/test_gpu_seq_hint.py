"""The first batch of launches of a sequenced BFS / SSSP / WCC run is sized by
the launches the previous run of the same algorithm on the same graph needed
(a launch after the run's end returns at once but still costs a few
microseconds).  The hint only changes how many launches are enqueued ahead,
so every result must equal the oracle's whatever it is: too high (a near
source after a far one) or too low (a far source after a near one, where the
run continues over further batches)."""
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


def test_repeated_runs_enqueue_fewer_launches(engine):
    g = gen.rmat(16, seed=61, weights=(1, 64))
    src = gen.max_degree_vertex(g)
    dg = engine.load(g)
    try:
        for algo, name, ref in [(sx.SX_BFS, "bfs", oracle.bfs_g(g, src)),
                                (sx.SX_SSSP, "sssp", oracle.sssp_g(g, src)),
                                (sx.SX_WCC, "wcc", oracle.wcc_g(g))]:
            launches = []
            for rep in range(3):
                announce(f"seq hint rmat16 {name} rep {rep}")
                out, st = run(engine, g, algo, src if algo != sx.SX_WCC else -1, dg=dg)
                np.testing.assert_array_equal(out, ref)
                launches.append(st["launches"])
            print(f"[seq-hint] rmat16 {name} launches {launches}", flush=True)
            # the first run enqueues 16 after the set-up launch; BFS and SSSP
            # on this graph need about ten, so the later runs enqueue less
            if algo != sx.SX_WCC:
                assert launches[1] < launches[0] and launches[2] < launches[0]
    finally:
        dg.close()


def test_hint_too_low_and_too_high(engine):
    n = 1500
    g = gen.from_edges(n, [(i, i + 1) for i in range(n - 1)], [1 + (i % 7) for i in range(n - 1)])
    dg = engine.load(g)
    try:
        for algo, name, oracle_fn in [(sx.SX_BFS, "bfs", oracle.bfs_g), (sx.SX_SSSP, "sssp", oracle.sssp_g)]:
            # middle (about n / 2 levels), then an end (about n: the hint is
            # too low), then the middle again (too high), then the end again
            for src in (n // 2, 0, n // 2, n - 1):
                announce(f"seq hint path-{n} {name} src={src}")
                out, _ = run(engine, g, algo, src, dg=dg)
                np.testing.assert_array_equal(out, oracle_fn(g, src))
    finally:
        dg.close()
