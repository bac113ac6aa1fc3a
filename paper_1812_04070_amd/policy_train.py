"""Train the per-iteration policy MLP on timings the engine itself measures.

    python -m paper_1812_04070_amd.policy_train [--out policy_mlp.json] [--quick]

1. Collect: for BFS and SSSP on the training workloads (R-MAT scale 16, the
   scale-22 graph, a 4096^2 grid with 10 % of edges deleted, and smaller R-MAT
   and grid graphs), `sx_policy_collect` times, before each iteration, six ways
   of running it from the same saved state (push on the online lists, push
   after a ballot rebuild with four bin-threshold pairs, pull).
2. Label: the fastest arm gives the pull target; among push arms, whether a
   ballot rebuild won; the thresholds of the fastest ballot arm give the two
   regression targets (log2).
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


def labels(arm_ms: np.ndarray):
    """targets [r, 4], weights [r, 4] from per-arm times (NaN = arm not
    possible).  The two classification heads are weighted by what a wrong
    choice costs on that record (relative time difference between the best
    push and the pull arm, and between the online and the best ballot arm,
    clipped to [0.05, 5]), so that iterations where the choice hardly
    matters do not outvote the ones where it does."""
    import paper_1812_04070_amd as sx
    r = arm_ms.shape[0]
    t = np.zeros((r, 4), dtype=np.float32)
    m = np.zeros((r, 4), dtype=np.float32)
    ms = np.where(np.isnan(arm_ms), np.inf, arm_ms)
    best = ms.argmin(1)
    t_push = ms[:, :5].min(1)
    t_pull = ms[:, 5]
    t[:, 0] = (t_pull < t_push)
    lo = np.minimum(t_push, t_pull)
    m[:, 0] = np.clip(np.abs(t_push - t_pull) / np.maximum(lo, 1e-6), 0.05, 5.0)
    t_on = ms[:, 0]
    t_bal = ms[:, 1:5].min(1)
    t[:, 1] = (t_bal < t_on)
    have_on = np.isfinite(t_on)
    lo = np.minimum(t_on, t_bal)
    w = np.clip(np.abs(t_on - t_bal) / np.maximum(lo, 1e-6), 0.05, 5.0)
    # without the online arm (after a pull or an overflow) the rebuild is forced
    m[:, 1] = np.where(have_on, w, 0.0)
    bb = 1 + ms[:, 1:5].argmin(1)
    th = np.array([sx.ARM_THRESHOLDS[k] for k in bb], dtype=np.float64)
    t[:, 2] = np.log2(th[:, 0])
    t[:, 3] = np.log2(th[:, 1])
    m[:, 2] = 1
    m[:, 3] = 1
    return t, m, best


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
    pick = np.where(y[:, 0] > 0, 5, np.where((y[:, 1] > 0) | ~np.isfinite(ms[:, 0]), 1 + ms[:, 1:5].argmin(1), 0))
    net_ms = float(ms[np.arange(len(ms)), pick].sum())
    summary = {
        "records": int(len(X)),
        "arm_wins": {str(k): int((best == k).sum()) for k in range(sx.SX_POLICY_ARMS)},
        "loss": hist,
        "train_acc_direction": acc_dir,
        "train_acc_filter": acc_flt,
        "best_arm_ms_total": float(ms.min(1).sum()),
        "network_arm_ms_total": net_ms,
        "workloads": sorted(set(tags.tolist())),
    }
    with open(args.out, "w") as f:
        json.dump({"params": [float(v) for v in P], "summary": summary}, f)
    print(json.dumps(summary))
    eng.close()


if __name__ == "__main__":
    main()
