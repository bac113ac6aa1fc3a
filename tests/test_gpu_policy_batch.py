"""GPU tests of the learned policy (MLP kernels against the fp64 oracle,
policy independence of the results, timing collection) and of the batched
multi-query mode (results identical to the oracle for every team size)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import mlp as ref
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


def _dev(a, eng):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(eng.device)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 8)).astype(np.float32)
    t = np.stack([rng.integers(0, 2, n), rng.integers(0, 2, n), rng.uniform(2, 7, n),
                  rng.uniform(7, 11, n)], 1).astype(np.float32)
    m = (rng.random((n, 4)) < 0.8).astype(np.float32)
    return x, t, m


@pytest.mark.parametrize("n,seed,scale", [(1, 1, 1.0), (1000, 1, 1.0), (4099, 7, 3.0)])
def test_mlp_forward_matches_oracle(engine, n, seed, scale):
    """sx_mlp_forward evaluates through mlp_eval_wave, the device function
    every in-kernel decision of the learned policy calls: element by element
    against the FP64 oracle."""
    import torch
    p = (ref.init_params(seed) * scale).astype(np.float32)
    p[-4:] = np.array([0.5, -0.25, 4.0, 9.0], dtype=np.float32)
    x, _, _ = _data(n, seed + 1)
    announce(f"mlp forward n={n}")
    Y = torch.empty((n, 4), dtype=torch.float32, device=engine.device)
    P, X = _dev(p, engine), _dev(x, engine)
    sx.sx_mlp_forward(engine.ctx, P.data_ptr(), X.data_ptr(), n, Y.data_ptr(), engine.stream())
    y_ref, _ = ref.forward(p.astype(np.float64), x.astype(np.float64))
    np.testing.assert_allclose(Y.cpu().numpy(), y_ref, rtol=1e-5, atol=1e-5 * np.abs(y_ref).max())


@pytest.mark.parametrize("n", [1, 37, 4096])
def test_mlp_grad_matches_oracle(engine, n):
    import torch
    p = ref.init_params(3).astype(np.float32)
    x, t, m = _data(n, 4)
    announce(f"mlp loss+grad n={n}")
    P, X, T, M = (_dev(v, engine) for v in (p, x, t, m))
    G = torch.zeros(ref.NPARAMS, dtype=torch.float32, device=engine.device)
    L = torch.zeros(1, dtype=torch.float32, device=engine.device)
    sx.sx_mlp_loss_grad(engine.ctx, P.data_ptr(), X.data_ptr(), T.data_ptr(), M.data_ptr(), n,
                        L.data_ptr(), G.data_ptr(), engine.stream())
    g_ref = ref.grad(p.astype(np.float64), x.astype(np.float64), t, m)
    l_ref = ref.loss(p.astype(np.float64), x.astype(np.float64), t, m)
    g = G.cpu().numpy().astype(np.float64)
    # element by element: FP32 per-sample arithmetic with compensated sums
    # over the samples; the absolute floor is relative to the largest entry
    np.testing.assert_allclose(g, g_ref, rtol=1e-4, atol=1e-6 * np.abs(g_ref).max())
    assert np.linalg.norm(g - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    assert abs(L.item() - l_ref) <= 1e-5 * abs(l_ref)


def test_mlp_adam_matches_oracle(engine):
    import torch
    rng = np.random.default_rng(5)
    p = ref.init_params(6).astype(np.float32)
    g = rng.normal(size=ref.NPARAMS).astype(np.float32) * 1e-2
    mo = rng.normal(size=ref.NPARAMS).astype(np.float32) * 1e-3
    vo = np.abs(rng.normal(size=ref.NPARAMS)).astype(np.float32) * 1e-5
    P, G, Mo, Vo = (_dev(v, engine) for v in (p, g, mo, vo))
    sx.sx_mlp_adam(engine.ctx, P.data_ptr(), G.data_ptr(), Mo.data_ptr(), Vo.data_ptr(), 3, 1e-3,
                   stream=engine.stream())
    p2, m2, v2 = ref.adam(p.astype(np.float64), g.astype(np.float64), mo.astype(np.float64),
                          vo.astype(np.float64), 3, lr=1e-3)
    np.testing.assert_allclose(P.cpu().numpy(), p2, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(Mo.cpu().numpy(), m2, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(Vo.cpu().numpy(), v2, rtol=1e-5, atol=1e-12)


FUSIONS = [sx.SX_FUSE_AUTO, sx.SX_SEQUENCED, sx.SX_FUSED, sx.SX_FUSED_ALL, sx.SX_UNFUSED]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_learned_policy_keeps_results_exact(engine, seed):
    """Any network -- here random ones -- changes only the schedule, in every
    arrangement, and for SSSP also with delta-stepping buckets (a learned
    pull drops them)."""
    p = (ref.init_params(seed) * 3.0).astype(np.float32)
    sx.sx_policy_load_mlp(engine.ctx, p)
    # R-MAT s16 has frontiers above the engine's consultation threshold (2^18
    # arcs), the grid none: both paths of the decision
    for name, g in [("rmat16", gen.rmat(16, seed=seed + 3, weights=(1, 64))),
                    ("grid64", gen.grid(64, 0.1, seed=seed, weights=(1, 1000)))]:
        src = gen.max_degree_vertex(g)
        dg = engine.load(g)
        ref_d, ref_x = oracle.bfs_g(g, src), oracle.sssp_g(g, src)
        for fused in FUSIONS:
            pol = sx.Policy(policy=sx.SX_POLICY_LEARNED, fused=fused)
            announce(f"learned {name} seed={seed} fused={fused}")
            d, st = run(engine, g, sx.SX_BFS, src, pol, dg=dg)
            np.testing.assert_array_equal(d, ref_d)
            if name == "rmat16":
                assert st["policy_evals"] >= 1, st
            x, st = run(engine, g, sx.SX_SSSP, src, pol, dg=dg)
            np.testing.assert_array_equal(x, ref_x)
            for delta in (40, 2000):
                announce(f"learned {name} seed={seed} fused={fused} delta={delta}")
                x, st = run(engine, g, sx.SX_SSSP, src, pol, dg=dg, sssp_delta=delta)
                np.testing.assert_array_equal(x, ref_x)
        dg.close()


@pytest.mark.parametrize("fused", FUSIONS)
def test_learned_decisions_match_oracle_network(engine, fused):
    """The decisions the engine takes with the network: the features and
    outputs of the last evaluation in a run are exported through the run
    statistics, and the outputs equal the FP64 oracle network on those
    features (device inference in the sequenced and persistent kernels,
    host inference in the one-phase arrangement)."""
    p = (ref.init_params(11) * 2.0).astype(np.float32)
    sx.sx_policy_load_mlp(engine.ctx, p)
    g = gen.rmat(16, seed=13, weights=(1, 64))
    src = gen.max_degree_vertex(g)
    dg = engine.load(g)
    for algo in (sx.SX_BFS, sx.SX_SSSP):
        announce(f"learned decisions algo={algo} fused={fused}")
        _, st = run(engine, g, algo, src, sx.Policy(policy=sx.SX_POLICY_LEARNED, fused=fused), dg=dg)
        assert st["policy_evals"] >= 1, st
        x = np.asarray(st["policy_x"], dtype=np.float64)[None, :]
        assert np.all(np.isfinite(x)) and 0.0 < x[0, 0] <= 1.0
        y_ref, _ = ref.forward(p.astype(np.float64), x)
        np.testing.assert_allclose(st["policy_y"], y_ref[0], rtol=1e-5, atol=1e-5 * np.abs(y_ref).max())
        _, sh = run(engine, g, algo, src, sx.Policy(fused=fused), dg=dg)
        assert sh["policy_evals"] == 0
    dg.close()


def test_policy_collect(engine):
    import torch
    g = gen.rmat(12, seed=2, weights=(1, 64))
    src = gen.max_degree_vertex(g)
    dg = engine.load(g)
    out = torch.empty(g.n, dtype=torch.int32, device=engine.device)
    for algo, ref_fn in [(sx.SX_BFS, oracle.bfs_g), (sx.SX_SSSP, oracle.sssp_g)]:
        announce(f"collect algo={algo}")
        f, a = sx.sx_policy_collect(engine.program(algo), dg.handle, src, out.data_ptr(), engine.stream())
        assert len(f) >= 3 and f.shape[1] == 8 and a.shape[1] == sx.SX_POLICY_ARMS
        assert np.all(np.isfinite(a[:, 1:])) and np.all(a[:, 1:] > 0)
        h = engine.to_host(dg, algo, out)
        np.testing.assert_array_equal(h, ref_fn(g, src))
    dg.close()


def _batch_graphs():
    return [gen.rmat(10, seed=21, weights=(1, 64)), gen.rmat(16, seed=22, weights=(1, 64)),
            gen.grid(48, 0.1, seed=23, weights=(1, 64)), gen.grid(100, 0.1, seed=24, weights=(1, 64)),
            gen.random_graph(300, 0.02, seed=25, weights=(1, 64))]


@pytest.mark.parametrize("team", [1, 4, 32])
@pytest.mark.parametrize("learned", [False, True])
def test_batch_matches_oracle(engine, team, learned):
    import torch
    graphs = _batch_graphs()
    dgs = [engine.load(g) for g in graphs]
    rng = np.random.default_rng(team)
    queries, refs, outs = [], [], []
    for i in range(24):
        gi = i % len(graphs)
        g = graphs[gi]
        cand = np.nonzero(g.out_degree() > 0)[0]
        s = int(rng.choice(cand))
        algo = sx.SX_BFS if i % 2 == 0 else sx.SX_SSSP
        out = torch.empty(g.n, dtype=torch.int32, device=engine.device)
        outs.append(out)
        queries.append((dgs[gi].handle, algo, s, out.data_ptr()))
        refs.append((gi, algo, oracle.bfs_g(g, s) if algo == sx.SX_BFS else oracle.sssp_g(g, s)))
    if learned:
        sx.sx_policy_load_mlp(engine.ctx, (ref.init_params(9) * 3.0).astype(np.float32))
    pol = sx.Policy(policy=sx.SX_POLICY_LEARNED if learned else sx.SX_POLICY_HEURISTIC).c()
    cfg = sx.sx_batch_config(team, 0, 0)
    announce(f"batch team={team} learned={learned}")
    ms, stats = sx.sx_run_batch(engine.ctx, queries, pol, cfg, engine.stream())
    assert ms > 0
    for (gi, algo, r), out in zip(refs, outs):
        h = engine.to_host(dgs[gi], algo, out)
        np.testing.assert_array_equal(h, r)
    for d in dgs:
        d.close()


def test_batch_autotune(engine):
    import torch
    graphs = _batch_graphs()[:3]
    dgs = [engine.load(g) for g in graphs]
    outs, queries = [], []
    for i, g in enumerate(graphs):
        out = torch.empty(g.n, dtype=torch.int32, device=engine.device)
        outs.append(out)
        queries.append((dgs[i].handle, sx.SX_SSSP, gen.max_degree_vertex(g), out.data_ptr()))
    announce("batch autotune")
    cfg, ms = sx.sx_batch_autotune(engine.ctx, queries, None, engine.stream())
    assert cfg["team_wgs"] in (1, 2, 4, 8, 16, 32) and ms > 0
    ms2, _ = sx.sx_run_batch(engine.ctx, queries, None, None, engine.stream())
    for i, g in enumerate(graphs):
        np.testing.assert_array_equal(engine.to_host(dgs[i], sx.SX_SSSP, outs[i]),
                                      oracle.sssp_g(g, gen.max_degree_vertex(g)))
    for d in dgs:
        d.close()


def _trained_params():
    import json
    import os
    path = os.path.join(os.path.dirname(sx.__file__), "policy_mlp.json")
    if not os.path.exists(path):
        pytest.skip("no trained policy (run python -m paper_1812_04070_amd.policy_train)")
    with open(path) as f:
        return np.asarray(json.load(f)["params"], dtype=np.float32)


def test_trained_policy_gain(engine):
    """What the trained network gains over the heuristic it replaces: BFS and
    SSSP device time on graphs of the training families (R-MAT and a grid
    with deleted edges, fresh seeds), heuristic vs learned policy, outputs
    identical.  On these workloads the heuristic runs within 0.6 % of the
    best arm per iteration (training records), so the network departs from
    it only with a confident logit and only on heavy iterations: the bound is
    no measurable loss (learned total within 3 % of the heuristic's, the
    run-to-run spread of these timings), not a gain."""
    sx.sx_policy_load_mlp(engine.ctx, _trained_params())
    heur, learned = sx.Policy(), sx.Policy(policy=sx.SX_POLICY_LEARNED)
    rows, tot_h, tot_l = [], 0.0, 0.0
    for name, g in [("rmat17", gen.rmat(17, seed=31, weights=(1, 64))),
                    ("rmat19", gen.rmat(19, seed=32, weights=(1, 64))),
                    ("grid1024", gen.grid(1024, 0.1, seed=33, weights=(1, 64), weight_seed=34))]:
        src = 0 if name.startswith("grid") else gen.max_degree_vertex(g)
        dg = engine.load(g)
        for algo, aname in [(sx.SX_BFS, "bfs"), (sx.SX_SSSP, "sssp")]:
            announce(f"trained-policy gain {name} {aname}")
            ts = {}
            outs = {}
            for pname, pol in [("heuristic", heur), ("learned", learned)]:
                times = []
                for _ in range(3):
                    h, st = run(engine, g, algo, src, pol, dg=dg)
                    times.append(st["device_ms"])
                ts[pname] = float(np.median(times))
                outs[pname] = h
            np.testing.assert_array_equal(outs["learned"], outs["heuristic"])
            rows.append((name, aname, ts["heuristic"], ts["learned"]))
            tot_h += ts["heuristic"]
            tot_l += ts["learned"]
        dg.close()
    for r in rows:
        print(f"[policy-gain] {r[0]:9s} {r[1]:4s} heuristic {r[2]:8.3f} ms  learned {r[3]:8.3f} ms  "
              f"gain {r[2] / r[3]:.3f}x", flush=True)
    print(f"[policy-gain] total heuristic {tot_h:.3f} ms learned {tot_l:.3f} ms gain {tot_h / tot_l:.3f}x",
          flush=True)
    assert tot_l <= 1.03 * tot_h
