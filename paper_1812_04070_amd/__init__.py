"""MI355X implementation of the ACC (Active-Compute-Combine) graph engine of
"SIMD-X: Programming and Processing of Graph Algorithms on GPUs" (Liu & Huang).

This module is the thin Python binding of ``libsimdx.so`` (C ABI declared in
``include/simdx.h``).  It only marshals arguments: every step of a run executes
in the library's HIP kernels.  PyTorch provides device memory and streams.
There is no fallback: if the library is not built, importing the binding's
functions raises.

Low-level names mirror the C ABI (``sx_ctx_create``, ``sx_graph_load``,
``sx_program_register``, ``sx_program_set_policy``, ``sx_run``,
``sx_read_vertices``, ...).  ``Engine`` wraps them for convenience.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsimdx.so")

# status codes
SX_OK, SX_EINVAL, SX_ENOMEM, SX_EHIP, SX_EUNSUPPORTED, SX_EDEADLOCK, SX_EOVERFLOW, SX_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
# graph flags
SX_UNDIRECTED, SX_DEVICE_PTRS, SX_VALIDATE, SX_REORDER = 1, 2, 4, 8
# algorithms
SX_BFS, SX_SSSP, SX_KCORE, SX_PAGERANK, SX_WCC, SX_BP = 0, 1, 2, 3, 4, 5
# policy enums
SX_DIR_AUTO, SX_DIR_PUSH, SX_DIR_PULL = 0, 1, 2
SX_FILTER_JIT, SX_FILTER_ONLINE, SX_FILTER_BALLOT = 0, 1, 2
SX_FUSE_AUTO, SX_FUSED, SX_UNFUSED, SX_SEQUENCED, SX_FUSED_ALL = 0, 1, 2, 3, 4
SX_POLICY_HEURISTIC, SX_POLICY_LEARNED = 0, 1

ALGOS = {"bfs": SX_BFS, "sssp": SX_SSSP, "kcore": SX_KCORE, "pagerank": SX_PAGERANK, "wcc": SX_WCC,
         "bp": SX_BP}

EXPORTED = [
    "sx_ctx_create", "sx_ctx_destroy", "sx_status_str", "sx_last_error",
    "sx_graph_load", "sx_graph_destroy", "sx_graph_info",
    "sx_program_register", "sx_program_destroy", "sx_program_set_policy",
    "sx_run", "sx_read_vertices", "sx_kernel_info_get", "sx_eq1_ctas",
    "sx_policy_load_mlp", "sx_mlp_forward", "sx_mlp_forward_host", "sx_mlp_loss_grad", "sx_mlp_adam",
    "sx_policy_collect", "sx_run_batch", "sx_batch_autotune",
    "sx_run_iterations", "sx_frontier_get", "sx_run_static",
]
SX_POLICY_ARMS = 6
ARM_THRESHOLDS = [None, (16, 256), (64, 256), (64, 1024), (256, 2048), None]
SX_MLP_NPARAMS = 1476


class sx_graph_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("in_offsets", ctypes.c_void_p),
                ("in_indices", ctypes.c_void_p), ("in_weights", ctypes.c_void_p),
                ("flags", ctypes.c_uint32)]


class sx_algo_params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("pr_damping", ctypes.c_float), ("pr_iters", ctypes.c_int32),
                ("sssp_delta", ctypes.c_uint32), ("kcore_k", ctypes.c_int32),
                ("pr_tol", ctypes.c_float), ("bp_kappa", ctypes.c_float), ("bp_iters", ctypes.c_int32)]


class sx_policy(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("filter", ctypes.c_int32),
                ("bin_small", ctypes.c_int32), ("bin_large", ctypes.c_int32),
                ("online_cap", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("policy", ctypes.c_int32), ("grid_wgs", ctypes.c_int32),
                ("watchdog_us", ctypes.c_int32), ("kcore_tail", ctypes.c_int32)]


class sx_run_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("pull_iters", ctypes.c_int32), ("ballot_iters", ctypes.c_int32),
                ("edges_inspected", ctypes.c_int64), ("vertex_expansions", ctypes.c_int64),
                ("device_ms", ctypes.c_double), ("scan_entries", ctypes.c_int64),
                ("barrier_wait_ms", ctypes.c_double), ("policy_evals", ctypes.c_int32),
                ("policy_x", ctypes.c_float * 8), ("policy_y", ctypes.c_float * 4)]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, ctypes.Array) else v
        return out


class sx_query(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("algo", ctypes.c_int), ("source", ctypes.c_int32),
                ("d_out", ctypes.c_void_p)]


class sx_batch_config(ctypes.Structure):
    _fields_ = [("team_wgs", ctypes.c_int32), ("bin_small", ctypes.c_int32), ("bin_large", ctypes.c_int32)]


class sx_kernel_info(ctypes.Structure):
    _fields_ = [("vgprs", ctypes.c_int32), ("sgprs", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("block", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("grid_wgs", ctypes.c_int32), ("cus", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsimdx.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1812_04070_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, P = ctypes.c_void_p, ctypes.POINTER
    sig = {
        "sx_ctx_create": ([ctypes.c_int, P(vp)], ctypes.c_int),
        "sx_ctx_destroy": ([vp], None),
        "sx_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "sx_last_error": ([], ctypes.c_char_p),
        "sx_graph_load": ([vp, P(sx_graph_desc), vp, P(vp)], ctypes.c_int),
        "sx_graph_destroy": ([vp], None),
        "sx_graph_info": ([vp, P(ctypes.c_int32), P(ctypes.c_int64), P(ctypes.c_int32), P(ctypes.c_int32)],
                          ctypes.c_int),
        "sx_program_register": ([vp, P(sx_algo_params), P(vp)], ctypes.c_int),
        "sx_program_destroy": ([vp], None),
        "sx_program_set_policy": ([vp, P(sx_policy)], ctypes.c_int),
        "sx_run": ([vp, vp, ctypes.c_int32, vp, vp, P(sx_run_stats)], ctypes.c_int),
        "sx_run_static": ([vp, P(sx_graph_desc), ctypes.c_int32, vp, vp, P(sx_run_stats)], ctypes.c_int),
        "sx_read_vertices": ([vp, ctypes.c_int, vp, vp, vp], ctypes.c_int),
        "sx_kernel_info_get": ([vp, ctypes.c_char_p, P(sx_kernel_info)], ctypes.c_int),
        "sx_eq1_ctas": ([ctypes.c_int32] * 4, ctypes.c_int32),
        "sx_policy_load_mlp": ([vp, vp, ctypes.c_int64], ctypes.c_int),
        "sx_mlp_forward": ([vp, vp, vp, ctypes.c_int32, vp, vp], ctypes.c_int),
        "sx_mlp_forward_host": ([vp, vp, ctypes.c_int32, vp], ctypes.c_int),
        "sx_mlp_loss_grad": ([vp, vp, vp, vp, vp, ctypes.c_int32, vp, vp, vp], ctypes.c_int),
        "sx_mlp_adam": ([vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                         ctypes.c_float, ctypes.c_float, vp], ctypes.c_int),
        "sx_policy_collect": ([vp, vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp, ctypes.c_int32,
                               P(ctypes.c_int32)], ctypes.c_int),
        "sx_run_batch": ([vp, P(sx_query), ctypes.c_int32, P(sx_policy), P(sx_batch_config), vp,
                          P(sx_run_stats), P(ctypes.c_double)], ctypes.c_int),
        "sx_batch_autotune": ([vp, P(sx_query), ctypes.c_int32, P(sx_policy), vp, P(sx_batch_config),
                               P(ctypes.c_double)], ctypes.c_int),
        "sx_run_iterations": ([vp, vp, ctypes.c_int32, vp, vp, ctypes.c_int32, P(sx_run_stats)], ctypes.c_int),
        "sx_frontier_get": ([vp, vp, vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32), vp,
                             ctypes.c_int64, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class SxError(RuntimeError):
    def __init__(self, status: int, what: str):
        L = lib()
        detail = L.sx_last_error().decode(errors="replace")
        super().__init__(f"{what}: {L.sx_status_str(status).decode()} ({status}): {detail}")
        self.status = status


def check(status: int, what: str) -> None:
    if status != SX_OK:
        raise SxError(status, what)


# ---------------------------------------------------------------------------
# Thin wrappers with the C names
# ---------------------------------------------------------------------------

def sx_status_str(status: int) -> str:
    return lib().sx_status_str(status).decode()


def sx_last_error() -> str:
    return lib().sx_last_error().decode(errors="replace")


def sx_graph_info(g) -> dict:
    n, m, d, w = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().sx_graph_info(g, ctypes.byref(n), ctypes.byref(m), ctypes.byref(d), ctypes.byref(w)),
          "sx_graph_info")
    return {"n": n.value, "m": m.value, "directed": bool(d.value), "weighted": bool(w.value)}


def sx_ctx_create(device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(lib().sx_ctx_create(device, ctypes.byref(h)), "sx_ctx_create")
    return h


def sx_ctx_destroy(ctx) -> None:
    lib().sx_ctx_destroy(ctx)


def sx_graph_load(ctx, desc: sx_graph_desc, stream: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(lib().sx_graph_load(ctx, ctypes.byref(desc), ctypes.c_void_p(stream), ctypes.byref(h)),
          "sx_graph_load")
    return h


def sx_graph_destroy(g) -> None:
    lib().sx_graph_destroy(g)


SX_DELTA_AUTO = 0xFFFFFFFF


def sx_program_register(ctx, algo: int, pr_damping: float = 0.85, pr_iters: int = 20, sssp_delta: int = 0,
                        kcore_k: int = 0, bp_kappa: float = 0.5, bp_iters: int = 10, pr_tol: float = 0.0):
    h = ctypes.c_void_p()
    p = sx_algo_params(algo, pr_damping, pr_iters, sssp_delta, kcore_k, pr_tol, bp_kappa, bp_iters)
    check(lib().sx_program_register(ctx, ctypes.byref(p), ctypes.byref(h)), "sx_program_register")
    return h


def sx_program_destroy(p) -> None:
    lib().sx_program_destroy(p)


def sx_program_set_policy(p, pol: sx_policy) -> None:
    check(lib().sx_program_set_policy(p, ctypes.byref(pol)), "sx_program_set_policy")


def sx_run(p, g, source: int, d_out_ptr: int, stream: int = 0) -> sx_run_stats:
    st = sx_run_stats()
    check(lib().sx_run(p, g, source, ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(stream),
                       ctypes.byref(st)), "sx_run")
    return st


def sx_run_static(p, desc: sx_graph_desc, source: int, d_out_ptr: int, stream: int = 0) -> sx_run_stats:
    st = sx_run_stats()
    check(lib().sx_run_static(p, ctypes.byref(desc), source, d_out_ptr, stream, ctypes.byref(st)),
          "sx_run_static")
    return st


def sx_run_iterations(p, g, source: int, d_out_ptr: int, iterations: int, stream: int = 0) -> sx_run_stats:
    st = sx_run_stats()
    check(lib().sx_run_iterations(p, g, source, ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(stream),
                                  iterations, ctypes.byref(st)), "sx_run_iterations")
    return st


def sx_frontier_get(g, cap: int, nwords: int = 0, stream: int = 0):
    """(vertices, bins, from_ballot, words) of the list left by sx_run_iterations."""
    v = np.zeros(max(cap, 1), dtype=np.int32)
    b = np.zeros(max(cap, 1), dtype=np.int32)
    w = np.zeros(max(nwords, 1), dtype=np.uint64)
    cnt, fb = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib().sx_frontier_get(g, v.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p), cap,
                                ctypes.byref(cnt), ctypes.byref(fb),
                                w.ctypes.data_as(ctypes.c_void_p) if nwords else None, nwords,
                                ctypes.c_void_p(stream)), "sx_frontier_get")
    k = min(cnt.value, cap)
    if cnt.value > cap:
        raise ValueError(f"list of {cnt.value} entries exceeds cap {cap}")
    return v[:k].copy(), b[:k].copy(), bool(fb.value), w[:nwords].copy()


def sx_read_vertices(g, algo: int, d_out_ptr: int, host: np.ndarray, stream: int = 0) -> None:
    check(lib().sx_read_vertices(g, algo, ctypes.c_void_p(d_out_ptr),
                                 host.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(stream)),
          "sx_read_vertices")


def sx_kernel_info_get(ctx, name: str) -> dict:
    ki = sx_kernel_info()
    check(lib().sx_kernel_info_get(ctx, name.encode(), ctypes.byref(ki)), "sx_kernel_info_get")
    return {k: getattr(ki, k) for k, _ in ki._fields_}


def sx_eq1_ctas(regs_per_sm: int, regs_per_thread: int, threads_per_wg: int, sms: int) -> int:
    return int(lib().sx_eq1_ctas(regs_per_sm, regs_per_thread, threads_per_wg, sms))


def sx_policy_load_mlp(ctx, params: np.ndarray) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    check(lib().sx_policy_load_mlp(ctx, p.ctypes.data_as(ctypes.c_void_p), p.size), "sx_policy_load_mlp")


def sx_mlp_forward(ctx, d_params: int, d_x: int, n: int, d_y: int, stream: int = 0) -> None:
    check(lib().sx_mlp_forward(ctx, ctypes.c_void_p(d_params), ctypes.c_void_p(d_x), n,
                               ctypes.c_void_p(d_y), ctypes.c_void_p(stream)), "sx_mlp_forward")


def sx_mlp_forward_host(params: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The network on the host (the one-phase arrangement's decisions)."""
    p = np.ascontiguousarray(params, dtype=np.float32)
    xx = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 8)
    y = np.empty((xx.shape[0], 4), dtype=np.float32)
    check(lib().sx_mlp_forward_host(p.ctypes.data_as(ctypes.c_void_p), xx.ctypes.data_as(ctypes.c_void_p),
                                    xx.shape[0], y.ctypes.data_as(ctypes.c_void_p)), "sx_mlp_forward_host")
    return y


def sx_mlp_loss_grad(ctx, d_params: int, d_x: int, d_t: int, d_mask: int, n: int, d_loss: int,
                     d_grad: int, stream: int = 0) -> None:
    check(lib().sx_mlp_loss_grad(ctx, *[ctypes.c_void_p(v) for v in (d_params, d_x, d_t, d_mask)], n,
                                 ctypes.c_void_p(d_loss), ctypes.c_void_p(d_grad), ctypes.c_void_p(stream)),
          "sx_mlp_loss_grad")


def sx_mlp_adam(ctx, d_params: int, d_grad: int, d_m: int, d_v: int, step: int, lr: float = 1e-3,
                beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream: int = 0) -> None:
    check(lib().sx_mlp_adam(ctx, *[ctypes.c_void_p(v) for v in (d_params, d_grad, d_m, d_v)], step, lr,
                            beta1, beta2, eps, ctypes.c_void_p(stream)), "sx_mlp_adam")


def sx_policy_collect(p, g, source: int, d_out_ptr: int, stream: int = 0, stride: int = 1,
                      max_records: int = 4096):
    """Per-iteration arm timings for policy training: returns (features [r, 8], arm_ms [r, 6])."""
    feats = np.zeros((max_records, 8), dtype=np.float32)
    arms = np.zeros((max_records, SX_POLICY_ARMS), dtype=np.float32)
    nrec = ctypes.c_int32(0)
    check(lib().sx_policy_collect(p, g, source, ctypes.c_void_p(d_out_ptr), ctypes.c_void_p(stream), stride,
                                  feats.ctypes.data_as(ctypes.c_void_p), arms.ctypes.data_as(ctypes.c_void_p),
                                  max_records, ctypes.byref(nrec)), "sx_policy_collect")
    return feats[:nrec.value].copy(), arms[:nrec.value].copy()


def sx_run_batch(ctx, queries, pol=None, cfg=None, stream: int = 0):
    """queries: list of (graph handle, algo, source, d_out pointer).  Returns
    (batch_ms, [per-query stats dicts])."""
    nq = len(queries)
    arr = (sx_query * max(nq, 1))(*[sx_query(g, a, s, o) for g, a, s, o in queries])
    stats = (sx_run_stats * max(nq, 1))()
    ms = ctypes.c_double(0.0)
    check(lib().sx_run_batch(ctx, arr, nq, ctypes.byref(pol) if pol is not None else None,
                             ctypes.byref(cfg) if cfg is not None else None, ctypes.c_void_p(stream),
                             stats, ctypes.byref(ms)), "sx_run_batch")
    return ms.value, [stats[i].as_dict() for i in range(nq)]


def sx_batch_autotune(ctx, queries, pol=None, stream: int = 0):
    nq = len(queries)
    arr = (sx_query * max(nq, 1))(*[sx_query(g, a, s, o) for g, a, s, o in queries])
    best = sx_batch_config()
    ms = ctypes.c_double(0.0)
    check(lib().sx_batch_autotune(ctx, arr, nq, ctypes.byref(pol) if pol is not None else None,
                                  ctypes.c_void_p(stream), ctypes.byref(best), ctypes.byref(ms)),
          "sx_batch_autotune")
    return {"team_wgs": best.team_wgs, "bin_small": best.bin_small, "bin_large": best.bin_large}, ms.value


# ---------------------------------------------------------------------------
# Convenience layer over torch device memory
# ---------------------------------------------------------------------------

@dataclass
class Policy:
    direction: int = SX_DIR_AUTO
    filter: int = SX_FILTER_JIT
    bin_small: int = 0
    bin_large: int = 0
    online_cap: int = 0
    fused: int = SX_FUSE_AUTO
    policy: int = SX_POLICY_HEURISTIC
    grid_wgs: int = 0
    watchdog_us: int = 0
    kcore_tail: int = 0

    def c(self) -> sx_policy:
        return sx_policy(self.direction, self.filter, self.bin_small, self.bin_large,
                         self.online_cap, self.fused, self.policy, self.grid_wgs, self.watchdog_us,
                         self.kcore_tail)


OUT_DTYPES = {SX_BFS: "int32", SX_SSSP: "uint32", SX_KCORE: "int32", SX_PAGERANK: "float32",
              SX_WCC: "int32", SX_BP: "float32"}


class DeviceGraph:
    """A host graph (paper_1812_04070_amd.gen.Graph) made resident through torch
    tensors and borrowed by the library (SX_DEVICE_PTRS)."""

    def __init__(self, engine: "Engine", g, validate: bool = False, reorder: bool = False):
        import torch
        self.engine = engine
        self.n, self.m = int(g.n), int(g.m)
        self.directed = bool(g.directed)
        dev = engine.device

        def up(a, dt):
            if a is None:
                return None
            return torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(dev)

        self._t = {
            "offsets": up(g.offsets, np.int32), "indices": up(g.indices, np.int32),
            "weights": up(g.weights, np.int32) if g.weights is not None else None,
        }
        if self.directed:
            self._t["in_offsets"] = up(g.in_offsets, np.int32)
            self._t["in_indices"] = up(g.in_indices, np.int32)
            self._t["in_weights"] = up(g.in_weights, np.int32) if g.in_weights is not None else None
        ptr = lambda k: (self._t[k].data_ptr() if self._t.get(k) is not None and self._t[k].numel() else
                         (self._t[k].data_ptr() if self._t.get(k) is not None else None))
        flags = SX_DEVICE_PTRS | (0 if self.directed else SX_UNDIRECTED) | (SX_REORDER if reorder else 0)
        desc = sx_graph_desc(self.n, self.m, ptr("offsets"), ptr("indices"), ptr("weights"),
                             ptr("in_offsets") if self.directed else None,
                             ptr("in_indices") if self.directed else None,
                             ptr("in_weights") if self.directed else None, flags)
        if validate:
            _validate_host(g)
        torch.cuda.synchronize(dev)
        self.handle = sx_graph_load(engine.ctx, desc, engine.stream())
        # the same borrowed arrays, as sx_run_static takes them
        self.desc = sx_graph_desc(self.n, self.m, ptr("offsets"), ptr("indices"), ptr("weights"),
                                  ptr("in_offsets") if self.directed else None,
                                  ptr("in_indices") if self.directed else None,
                                  ptr("in_weights") if self.directed else None,
                                  flags & ~SX_REORDER)

    def close(self):
        if getattr(self, "handle", None):
            sx_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _validate_host(g):
    off = g.offsets.astype(np.int64)
    if off[0] != 0 or np.any(np.diff(off) < 0) or off[-1] != g.m:
        raise ValueError("bad CSR offsets")
    if g.m and (g.indices.min() < 0 or g.indices.max() >= g.n):
        raise ValueError("CSR index out of range")


class Engine:
    """One HIP device: a context plus one program per algorithm."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        lib()
        self.device = torch.device("cuda", device)
        self.ctx = sx_ctx_create(device)
        self.programs = {}

    def stream(self) -> int:
        import torch
        return torch.cuda.current_stream(self.device).cuda_stream

    def program(self, algo: int, pr_damping: float = 0.85, pr_iters: int = 20, sssp_delta: int = 0,
                kcore_k: int = 0, bp_kappa: float = 0.5, bp_iters: int = 10, pr_tol: float = 0.0):
        key = (algo, pr_damping, pr_iters, sssp_delta, kcore_k, bp_kappa, bp_iters, pr_tol)
        if key not in self.programs:
            self.programs[key] = sx_program_register(self.ctx, algo, pr_damping, pr_iters, sssp_delta, kcore_k,
                                                     bp_kappa, bp_iters, pr_tol)
        return self.programs[key]

    def load(self, g, validate: bool = False, reorder: bool = False) -> DeviceGraph:
        """Make `g` resident.  reorder: the library renumbers the vertices by
        decreasing degree (SX_REORDER); runs still take and return original ids."""
        return DeviceGraph(self, g, validate, reorder)

    def run(self, dg: DeviceGraph, algo: int, source: int = -1, policy: Optional[Policy] = None,
            out=None, pr_damping: float = 0.85, pr_iters: int = 20, sssp_delta: int = 0, kcore_k: int = 0,
            prior=None, bp_kappa: float = 0.5, bp_iters: int = 10, pr_tol: float = 0.0):
        """Run and return (torch device tensor, stats dict).  sssp_delta: SSSP
        bucket width of delta-stepping (0 = none); kcore_k: membership in the
        k-core instead of the decomposition (k > 0).  SX_BP: `prior` (n
        floats in (0, 1), host or device) is copied into the output array,
        which the run turns into the beliefs (or pass `out` already holding
        the priors)."""
        import torch
        p = self.program(algo, pr_damping, pr_iters, sssp_delta, kcore_k, bp_kappa, bp_iters, pr_tol)
        sx_program_set_policy(p, (policy or Policy()).c())
        if algo == SX_BP and prior is not None:
            t = torch.as_tensor(np.ascontiguousarray(prior, dtype=np.float32)
                                if isinstance(prior, np.ndarray) else prior)
            out = t.to(device=self.device, dtype=torch.float32).clone() if out is None else out.copy_(t)
            if dg.n == 0:
                out = torch.empty(1, dtype=torch.float32, device=self.device)
        elif algo == SX_BP and out is None:
            raise ValueError("SX_BP needs the priors (prior= or out=)")
        if out is None:
            dt = {SX_PAGERANK: torch.float32}.get(algo, torch.int32)
            out = torch.empty(max(dg.n, 1), dtype=dt, device=self.device)
        st = sx_run(p, dg.handle, source, out.data_ptr(), self.stream())
        return out[:dg.n], st.as_dict()

    def run_static(self, dg: DeviceGraph, algo: int, source: int = -1, policy: Optional[Policy] = None,
                   out=None, sssp_delta: int = 0):
        """sx_run_static on dg's device arrays: the run's workspace is the
        library's static array (nothing allocated by the call); returns
        (torch device tensor, stats dict) like run()."""
        import torch
        p = self.program(algo, sssp_delta=sssp_delta)
        sx_program_set_policy(p, (policy or Policy()).c())
        if out is None:
            out = torch.empty(max(dg.n, 1), dtype=torch.int32, device=self.device)
        st = sx_run_static(p, dg.desc, source, out.data_ptr(), self.stream())
        return out[:dg.n], st.as_dict()

    def to_host(self, dg: DeviceGraph, algo: int, out) -> np.ndarray:
        h = np.empty(dg.n, dtype=OUT_DTYPES[algo])
        if dg.n:
            sx_read_vertices(dg.handle, algo, out.data_ptr(), h, self.stream())
        return h

    def kernel_info(self, name: str) -> dict:
        return sx_kernel_info_get(self.ctx, name)

    def close(self):
        for p in self.programs.values():
            sx_program_destroy(p)
        self.programs = {}
        if self.ctx:
            sx_ctx_destroy(self.ctx)
            self.ctx = None
