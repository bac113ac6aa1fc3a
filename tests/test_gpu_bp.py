"""Belief propagation (SX_BP) against the FP64 oracle: the beliefs after a
fixed number of synchronous sum-product iterations, FP32 on the device.

Tolerance: relative L1 <= 1e-5 and every belief within 2e-5.  Each term
atanh(c q) and the final tanh / logistic carry a few FP32 roundings
(~1e-7 relative), the neighbour sums are compensated (TwoSum), and the
update is a contraction with factor about kappa <= 0.9, so the errors of
earlier iterations shrink instead of growing: the expected deviation is
~1e-6; the bound leaves a factor of ten."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1812_04070_amd as sx
from paper_1812_04070_amd import gen
from tests.gpu_util import announce, rel_l1

pytestmark = pytest.mark.gpu

TOL_L1, TOL_ABS = 1e-5, 2e-5


@pytest.fixture(scope="module")
def engine():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = sx.Engine(0)
    yield e
    e.close()


def _check(engine, dg, g, prior, kappa, iters, pol=None):
    out, st = engine.run(dg, sx.SX_BP, -1, pol, prior=prior, bp_kappa=kappa, bp_iters=iters)
    got = engine.to_host(dg, sx.SX_BP, out).astype(np.float64)
    ref = oracle.bp_g(g, prior.astype(np.float64), kappa, iters)
    assert rel_l1(got, ref) <= TOL_L1, rel_l1(got, ref)
    assert np.abs(got - ref).max() <= TOL_ABS, np.abs(got - ref).max()
    return st


GRAPHS = [
    ("er-9", lambda: gen.random_graph(9, 0.4, seed=1, weights=(1, 64))),
    ("er-300-unweighted", lambda: gen.random_graph(300, 0.05, seed=3)),
    ("rmat12", lambda: gen.rmat(12, seed=6, weights=(1, 64))),
    ("rmat14", lambda: gen.rmat(14, seed=9, weights=(1, 64))),
    ("grid-60", lambda: gen.grid(60, 0.1, seed=7, weights=(1, 64))),
    ("star-3000", lambda: gen.from_edges(3001, [(0, i) for i in range(1, 3001)], [1 + i % 64 for i in range(3000)])),
    ("edgeless-50", lambda: gen.from_edges(50, [], [])),
]
POLICIES = [("default", None), ("tiny-bins", sx.Policy(bin_small=4, bin_large=8)),
            ("small-grid", sx.Policy(grid_wgs=8))]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_bp_small(engine, name, make):
    g = make()
    prior = gen.bp_priors(g.n, seed=g.n)
    dg = engine.load(g)
    for kappa, iters in ((0.0, 3), (0.5, 1), (0.5, 10), (0.9, 25)):
        for pname, pol in POLICIES:
            announce(f"bp {name} kappa={kappa} iters={iters} {pname}")
            st = _check(engine, dg, g, prior, kappa, iters, pol)
            assert st["iterations"] == iters
    dg.close()


def test_bp_reordered_and_zero_iterations(engine):
    g = gen.rmat(15, seed=4, weights=(1, 64))
    prior = gen.bp_priors(g.n, seed=2)
    dr = engine.load(g, reorder=True)
    announce("bp rmat15 reordered")
    _check(engine, dr, g, prior, 0.7, 8)
    announce("bp zero iterations")
    out, _ = engine.run(dr, sx.SX_BP, -1, prior=prior, bp_iters=0)
    np.testing.assert_array_equal(engine.to_host(dr, sx.SX_BP, out), prior)
    dr.close()


def test_bp_rejects(engine):
    g = gen.rmat(10, seed=1, weights=(1, 64))
    dg = engine.load(g)
    bad = gen.bp_priors(g.n, seed=1)
    bad[17] = 1.0
    announce("bp prior outside (0, 1)")
    with pytest.raises(sx.SxError) as ei:
        engine.run(dg, sx.SX_BP, -1, prior=bad)
    assert ei.value.status == sx.SX_EINVAL
    # the engine runs normally afterwards
    _check(engine, dg, g, gen.bp_priors(g.n, seed=1), 0.5, 5)
    for kappa, iters in ((1.0, 5), (-0.1, 5), (0.5, -1)):
        with pytest.raises(sx.SxError) as ei:
            sx.sx_program_register(engine.ctx, sx.SX_BP, bp_kappa=kappa, bp_iters=iters)
        assert ei.value.status == sx.SX_EINVAL
    dg.close()
    gd = gen.random_graph(40, 0.1, seed=2, directed=True, weights=(1, 64))
    dd = engine.load(gd)
    with pytest.raises(sx.SxError) as ei:
        engine.run(dd, sx.SX_BP, -1, prior=gen.bp_priors(gd.n, seed=3))
    assert ei.value.status == sx.SX_EUNSUPPORTED
    dd.close()


def test_bp_rmat20(engine):
    g = gen.rmat(20, seed=12, weights=(1, 64))
    prior = gen.bp_priors(g.n, seed=20)
    dg = engine.load(g)
    announce("bp rmat20 kappa=0.5 iters=10")
    _check(engine, dg, g, prior, 0.5, 10)
    dg.close()
