"""Train the per-iteration policy MLP on timings the engine itself measures.

    python -m paper_1812_04070_amd.policy_train [--out policy_mlp.json] [--quick]

1. Collect: for BFS and SSSP on the training workloads (R-MAT scale 16, the
   scale-22 graph, a 4096^2 grid with 10 % of edges deleted, and smaller R-MAT
   and grid graphs), `sx_policy_collect` times, before each iteration, six ways
   of running it from the same saved state (push on the online lists, push
   after a ballot rebuild with four bin-threshold pairs, pull).
2. Label: the heuristic's own arm, unless another arm is more than 10 %
   faster on that record (then that arm): its direction, filter and -- for a
   ballot arm -- bin thresholds (log2) are the targets; elsewhere the
   heuristic's thresholds.
3. Train on the GPU with the library's own kernels (sx_mlp_loss_grad +
   sx_mlp_adam), full batch.
4. Write the parameters (1,476 floats) and the training summary as JSON.

Everything runs through the C ABI; torch only holds device memory.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_BINS = (64, 512)        # the heuristic's bin thresholds
POLICY_MIN_ARCS = 1 << 18       # the engine's kPolicyMinArcs (sx_policy.hpp)
DEVIATE_MARGIN = 0.10           # depart from the heuristic's arm only if >10 % faster
POLICY_MARGIN = 4.0             # the engine's kPolicyMargin (logit units, sx_policy.hpp)
DEFAULT_OUT = os.path.join(HERE, "policy_mlp.json")


def training_graphs(quick: bool):
    from . import gen
    gs = [("rmat16", lambda: gen.workload_graph("rmat16")),
          ("rmat14s11", lambda: gen.rmat(14, seed=11, weights=(1, 64))),
          ("rmat18s12", lambda: gen.rmat(18, seed=12, weights=(1, 64))),
          ("grid512", lambda: gen.grid(512, 0.1, seed=13, weights=(1, 64), weight_seed=14))]
    if not quick:
        gs += [("rmat22", lambda: gen.workload_graph("rmat22")),
               ("grid4096", lambda: gen.workload_graph("grid4096")),
               ("rmat20s15", lambda: gen.rmat(20, seed=15, weights=(1, 64)))]
    return gs


def labels(arm_ms: np.ndarray, margin: float = None):
    """targets [r, 4], weights [r, 4] from per-arm times (NaN = arm not
    possible).  The target of a record is the heuristic's own arm unless
    another arm is faster by more than `margin` (relative): the network is
    to depart from the heuristic only where the timings say that pays, by
    more than its in-kernel evaluation and the timing noise.  The two
    classification heads are weighted by what a wrong choice costs on that
    record (relative time difference between the best push and the pull
    arm, and between the online and the best ballot arm, clipped to
    [0.05, 5]), so that iterations where the choice hardly matters do not
    outvote the ones where it does.  Bin thresholds: the chosen ballot arm's
    where the target is a ballot arm, else the heuristic's (64, 512) -- the
    network's thresholds also bin the online lists, which no arm timed with
    other thresholds (targets taken from the best ballot arm regardless
    cost the online pushes 5-18 % with 16 / 256)."""
    import paper_1812_04070_amd as sx
    if margin is None:
        margin = DEVIATE_MARGIN
    r = arm_ms.shape[0]
    rows = np.arange(r)
    t = np.zeros((r, 4), dtype=np.float32)
    m = np.zeros((r, 4), dtype=np.float32)
    ms = np.where(np.isnan(arm_ms), np.inf, arm_ms)
    best = ms.argmin(1)
    harm = heuristic_arm(arm_ms)
    dev = ms[rows, best] < (1.0 - margin) * ms[rows, harm]
    target = np.where(dev, best, harm)
    t[:, 0] = target == 5
    t_push = ms[:, :5].min(1)
    t_pull = ms[:, 5]
    lo = np.minimum(t_push, t_pull)
    m[:, 0] = np.clip(np.abs(t_push - t_pull) / np.maximum(lo, 1e-6), 0.05, 5.0)
    t[:, 1] = (target >= 1) & (target <= 4)
    t_on = ms[:, 0]
    t_bal = ms[:, 1:5].min(1)
    have_on = np.isfinite(t_on)
    lo = np.minimum(t_on, t_bal)
    w = np.clip(np.abs(t_on - t_bal) / np.maximum(lo, 1e-6), 0.05, 5.0)
    # without the online arm (after a pull) the filter head is not used
    m[:, 1] = np.where(have_on, w, 0.0)
    ballot = (target >= 1) & (target <= 4)
    th = np.array([sx.ARM_THRESHOLDS[k] if 1 <= k <= 4 else DEFAULT_BINS for k in target], dtype=np.float64)
    t[:, 2] = np.where(ballot, np.log2(th[:, 0]), np.log2(DEFAULT_BINS[0]))
    t[:, 3] = np.where(ballot, np.log2(th[:, 1]), np.log2(DEFAULT_BINS[1]))
    m[:, 2] = 1
    m[:, 3] = 1
    return t, m, best


def heuristic_arm(arm_ms: np.ndarray) -> np.ndarray:
    """The arm the heuristic itself runs for each record: the pull (arm 5)
    where it was pulling -- the only case in which the collector marks the
    online push (arm 0) unavailable -- else the push of its own lists (arm
    0: the online lists, or the ballot rebuild it made after an overflow)."""
    return np.where(np.isnan(arm_ms[:, 0]), 5, 0)


def collect(eng, quick: bool, log=print):
    import torch
    import paper_1812_04070_amd as sx
    from . import gen
    feats, arms, tags = [], [], []
    rng = np.random.default_rng(7)
    for name, make in training_graphs(quick):
        g = make()
        dg = eng.load(g)
        deg = g.out_degree()
        cand = np.nonzero(deg > 0)[0]
        sources = [gen.max_degree_vertex(g)] + [int(v) for v in rng.choice(cand, 2, replace=False)]
        if name.startswith("grid"):
            sources = [0]
        stride = max(1, int(math.sqrt(g.n) / 16)) if name.startswith("grid") else 1
        out = torch.empty(g.n, dtype=torch.int32, device=eng.device)
        for algo, aname in [(sx.SX_BFS, "bfs"), (sx.SX_SSSP, "sssp")]:
            p = eng.program(algo)
            for s in sources:
                t0 = time.perf_counter()
                f, a = sx.sx_policy_collect(p, dg.handle, s, out.data_ptr(), eng.stream(), stride=stride,
                                            max_records=4096)
                feats.append(f)
                arms.append(a)
                tags += [f"{name}/{aname}"] * len(f)
                log(f"[collect] {name} {aname} src={s}: {len(f)} records in {time.perf_counter()-t0:.1f}s")
        dg.close()
    return np.concatenate(feats), np.concatenate(arms), np.array(tags)


def train(eng, X: np.ndarray, T: np.ndarray, M: np.ndarray, steps: int = 1500, lr: float = 3e-3,
          seed: int = 0, log=print):
    import torch
    import paper_1812_04070_amd as sx
    rng = np.random.default_rng(seed)
    p0 = np.zeros(sx.SX_MLP_NPARAMS, dtype=np.float32)
    # He-uniform weights, zero biases (layout W1, b1, W2, b2, W3, b3)
    o = 0
    for rows, cols in [(32, 8), (32, 32), (4, 32)]:
        lim = math.sqrt(6.0 / cols)
        p0[o:o + rows * cols] = rng.uniform(-lim, lim, rows * cols)
        o += rows * cols + rows
    dev = eng.device
    P = torch.from_numpy(p0).to(dev)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(dev)
    Md = torch.from_numpy(np.ascontiguousarray(M, dtype=np.float32)).to(dev)
    G = torch.zeros_like(P)
    Mo = torch.zeros_like(P)
    Vo = torch.zeros_like(P)
    L = torch.zeros(1, dtype=torch.float32, device=dev)
    n = X.shape[0]
    st = eng.stream()
    hist = []
    for step in range(1, steps + 1):
        sx.sx_mlp_loss_grad(eng.ctx, P.data_ptr(), Xd.data_ptr(), Td.data_ptr(), Md.data_ptr(), n,
                            L.data_ptr(), G.data_ptr(), st)
        sx.sx_mlp_adam(eng.ctx, P.data_ptr(), G.data_ptr(), Mo.data_ptr(), Vo.data_ptr(), step, lr,
                       stream=st)
        if step == 1 or step % 250 == 0:
            hist.append((step, float(L.item())))
            log(f"[train] step {step} loss {hist[-1][1]:.4f}")
    torch.cuda.synchronize()
    return P.cpu().numpy(), hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--save-data", default=None, help="write the collected records (.npz)")
    ap.add_argument("--data", default=None, help="train on records saved by --save-data")
    args = ap.parse_args()
    import paper_1812_04070_amd as sx
    eng = sx.Engine(0)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    if args.data:
        z = np.load(args.data)
        X, A, tags = z["X"], z["A"], z["tags"]
    else:
        X, A, tags = collect(eng, args.quick, log)
    if args.save_data:
        np.savez(args.save_data, X=X, A=A, tags=tags)
    T, M, best = labels(A)
    P, hist = train(eng, X, T, M, steps=args.steps, log=log)
    # training accuracy of the direction / filter heads
    import torch
    Y = torch.empty((len(X), 4), dtype=torch.float32, device=eng.device)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(eng.device)
    Pd = torch.from_numpy(P).to(eng.device)
    sx.sx_mlp_forward(eng.ctx, Pd.data_ptr(), Xd.data_ptr(), len(X), Y.data_ptr(), eng.stream())
    y = Y.cpu().numpy()
    acc_dir = float(((y[:, 0] > 0) == (T[:, 0] > 0.5)).mean())
    sel = M[:, 1] > 0
    acc_flt = float(((y[sel, 1] > 0) == (T[sel, 1] > 0.5)).mean()) if sel.any() else float("nan")
    ms = np.where(np.isnan(A), np.inf, A)
    # time of the arms the network picks, against the best arm and the arm
    # the heuristic rule picks (push on the online lists unless pulling)
    # the arms the deployed network picks: the engine consults it only for
    # frontiers of POLICY_MIN_ARCS arcs or more (feature 1 = log2(1 + arcs)
    # / 32), and a choice departs from the heuristic's only when its logit
    # leans the other way by more than the margin
    harm = heuristic_arm(A)
    consult = np.exp2(32.0 * X[:, 1]) - 1.0 >= POLICY_MIN_ARCS
    rows = np.arange(len(ms))
    heur_ms = float(ms[rows, harm].sum())

    def picks(tau):
        h_pull = harm == 5
        n_pull = y[:, 0] + np.where(h_pull, tau, -tau) > 0
        n_ballot = ~n_pull & (harm == 0) & (y[:, 1] - tau > 0)
        th = np.stack([np.clip(np.rint(y[:, 2]), 2, 8), np.clip(np.rint(y[:, 3]), 6, 12)], 1)
        arms_th = np.log2(np.array(sx.ARM_THRESHOLDS[1:5], dtype=np.float64))
        near = 1 + np.abs(th[:, None, :] - arms_th[None, :, :]).sum(2).argmin(1)
        # a push after the heuristic's pull: its lists are rebuilt (the
        # collector has no online arm there); counted as the (64, 256) rebuild
        pk = np.where(n_pull, 5, np.where(n_ballot, near, np.where(harm == 5, 2, 0)))
        return np.where(consult, pk, harm)

    margins = {f"{tau:g}": float(ms[rows, picks(tau)].sum()) for tau in (0.0, 0.5, 1.0, 2.0, 4.0)}
    pick = picks(POLICY_MARGIN)
    net_ms = float(ms[rows, pick].sum())
    summary = {
        "records": int(len(X)),
        "arm_wins": {str(k): int((best == k).sum()) for k in range(sx.SX_POLICY_ARMS)},
        "loss": hist,
        "train_acc_direction": acc_dir,
        "train_acc_filter": acc_flt,
        "best_arm_ms_total": float(ms.min(1).sum()),
        "heuristic_arm_ms_total": heur_ms,
        "network_arm_ms_total": net_ms,
        "network_arm_ms_total_by_margin": margins,
        "records_network_consulted": int(consult.sum()),
        "records_network_differs_from_heuristic": int((pick != harm).sum()),
        "workloads": sorted(set(tags.tolist())),
    }
    with open(args.out, "w") as f:
        json.dump({"params": [float(v) for v in P], "summary": summary}, f)
    print(json.dumps(summary))
    eng.close()


if __name__ == "__main__":
    main()
