"""The C-ABI library loads and exports every symbol include/simdx.h declares;
host-only arithmetic (no GPU needed)."""
from __future__ import annotations

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "simdx.h")
LIB = os.path.join(ROOT, "paper_1812_04070_amd", "libsimdx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ["sx_ctx_create", "sx_graph_load", "sx_program_register", "sx_run",
                 "sx_read_vertices", "sx_program_set_policy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libsimdx.so not built")
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB]).decode()
    exported = set(re.findall(r" T (sx_[a-z0-9_]+)$", out, flags=re.M))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_1812_04070_amd as sx
    assert sorted(sx.EXPORTED) == declared_functions()
    for name in sx.EXPORTED:
        assert hasattr(sx, name)


def test_eq1_worked_example():
    """Section 5, Eq. 1: 110 registers per thread, 128 threads per CTA, 65,536
    registers per SMX and 15 SMX give 60 CTAs (4 per SMX; the text writes ceil
    but its result is the floor)."""
    if not os.path.exists(LIB):
        pytest.skip("libsimdx.so not built")
    import paper_1812_04070_amd as sx
    assert sx.sx_eq1_ctas(65536, 110, 128, 15) == 60
    assert sx.sx_eq1_ctas(65536, 48, 128, 15) == 150
    assert sx.sx_eq1_ctas(0, 1, 1, 1) == -1


def test_errors_without_device():
    """With no HIP device the context call fails cleanly with SX_EHIP or SX_EINVAL."""
    if not os.path.exists(LIB):
        pytest.skip("libsimdx.so not built")
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("device present")
    except Exception:
        pass
    import ctypes
    import paper_1812_04070_amd as sx
    h = ctypes.c_void_p()
    rc = sx.lib().sx_ctx_create(0, ctypes.byref(h))
    assert rc in (sx.SX_EHIP, sx.SX_EINVAL)
    assert sx.lib().sx_last_error()
    assert sx.lib().sx_status_str(sx.SX_EDEADLOCK)


def test_struct_layouts_match_binding(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program built against include/simdx.h prints them), and the
    binding's constants equal the header's."""
    import ctypes
    import shutil
    import paper_1812_04070_amd as sx
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    structs = [sx.sx_graph_desc, sx.sx_algo_params, sx.sx_policy, sx.sx_run_stats, sx.sx_query,
               sx.sx_batch_config, sx.sx_kernel_info]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "simdx.h"', 'int main(void) {']
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines.append('  printf("SX_DELTA_AUTO %u\\n", (unsigned)SX_DELTA_AUTO);')
    lines.append('  return 0;\n}')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for field, _ in st._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(st, field).offset, f"{name}.{field}"
    assert int(got["SX_DELTA_AUTO"]) == sx.SX_DELTA_AUTO


def test_host_inference_matches_oracle():
    """sx_mlp_forward_host (the network as the one-phase arrangement's host
    decisions evaluate it) against the FP64 oracle's forward pass."""
    if not os.path.exists(LIB):
        pytest.skip("libsimdx.so not built")
    import numpy as np
    import paper_1812_04070_amd as sx
    from oracle import mlp
    rng = np.random.default_rng(4)
    for seed, scale in [(0, 1.0), (1, 3.0), (2, 0.2)]:
        p = (mlp.init_params(seed) * scale).astype(np.float32)
        p[mlp.NPARAMS - 4:] = rng.normal(size=4)
        x = rng.normal(size=(300, 8)).astype(np.float32)
        y = sx.sx_mlp_forward_host(p, x)
        ref, _ = mlp.forward(p.astype(np.float64), x.astype(np.float64))
        np.testing.assert_allclose(y, ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())
    assert sx.lib().sx_mlp_forward_host(None, None, 1, None) == sx.SX_EINVAL
