"""Shared set-up for the GPU tests: one engine per session, named cases."""
from __future__ import annotations

import sys

import numpy as np

import paper_1812_04070_amd as sx


def announce(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def run(engine, g, algo, source=-1, policy=None, dg=None, **kw):
    own = dg is None
    if own:
        dg = engine.load(g)
    out, st = engine.run(dg, algo, source, policy, **kw)
    host = engine.to_host(dg, algo, out)
    if own:
        dg.close()
    return host, st


ARMS = [
    ("auto-jit", sx.Policy()),
    ("pull-seq", sx.Policy(direction=sx.SX_DIR_PULL, fused=sx.SX_SEQUENCED)),
    ("push-ballot-seq", sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_BALLOT, fused=sx.SX_SEQUENCED)),
    ("auto-jit-fused", sx.Policy(fused=sx.SX_FUSED)),
    ("push-online-fused", sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_ONLINE, fused=sx.SX_FUSED)),
    ("push-ballot-fused", sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_BALLOT, fused=sx.SX_FUSED)),
    ("pull-fused", sx.Policy(direction=sx.SX_DIR_PULL, fused=sx.SX_FUSED)),
    ("auto-jit-unfused", sx.Policy(fused=sx.SX_UNFUSED)),
    ("pull-unfused", sx.Policy(direction=sx.SX_DIR_PULL, fused=sx.SX_UNFUSED)),
    ("push-ballot-unfused", sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_BALLOT, fused=sx.SX_UNFUSED)),
    ("tiny-bins-jit", sx.Policy(bin_small=4, bin_large=8, online_cap=1)),
    ("wide-bins-small-grid", sx.Policy(bin_small=128, bin_large=2048, grid_wgs=8)),
]


def rel_l1(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).sum() / np.abs(ref).sum())
