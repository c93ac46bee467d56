"""CPU checks of the C ABI: the library loads, exports every function that
include/ndgp.h declares, its structs have the layout the Python binding
assumes, and argument checks fail cleanly before any GPU work."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from paper_1511_08200_amd import ndgp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ndgp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ndgp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ndgp.LIB_PATH):
        from paper_1511_08200_amd import build
        build.build()
    return ndgp.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "ndgp_solve" in names and "ndgp_residual" in names and "ndgp_force" in names
    for name in names:
        assert hasattr(L, name), f"{name} declared in ndgp.h but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", ndgp.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ndgp_\w+)", out))
    assert set(names) <= exported


def test_version_and_beta(L):
    assert L.ndgp_version() == 3
    for rc in (0.5, 1.0, 2.0, 5.0):
        assert ndgp.beta_lcdm(1.0, 0.3, rc) == pytest.approx(1 + 1.7 * rc, rel=1e-14)
    # a < 1: against Eq. (beta) with a numerical Hdot
    import math
    om, a, rc = 0.269, 0.5, 1.0
    H = lambda x: math.sqrt(om / x**3 + 1 - om)
    eps = 1e-6
    hdot = (H(a + eps) - H(a - eps)) / (2 * eps) * a * H(a)
    assert ndgp.beta_lcdm(a, om, rc) == pytest.approx(1 + 2 * H(a) * rc * (1 + hdot / (3 * H(a) ** 2)),
                                                      rel=1e-9)


def test_struct_layout_matches_c(L, tmp_path):
    """sizeof/offsetof from the C compiler against the ctypes mirrors."""
    src = tmp_path / "layout.c"
    fields = {
        "ndgp_grid": [f for f, _ in ndgp._Grid._fields_],
        "ndgp_params": [f for f, _ in ndgp._Params._fields_],
        "ndgp_report": [f for f, _ in ndgp._Report._fields_],
        "ndgp_geff_level": [f for f, _ in ndgp._GeffLevel._fields_],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ndgp.h"', "int main(void){"]
    for s, fs in fields.items():
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            parts = line.split()
            got[tuple(parts[:-1])] = int(parts[-1])
    for s, cls in (("ndgp_grid", ndgp._Grid), ("ndgp_params", ndgp._Params),
                   ("ndgp_report", ndgp._Report), ("ndgp_geff_level", ndgp._GeffLevel)):
        assert got[(s, "size")] == ctypes.sizeof(cls)
        for f, _ in cls._fields_:
            assert got[(s, f)] == getattr(cls, f).offset, (s, f)


def _args(n=32, h=1e-3, **kw):
    g = ndgp._Grid()
    g.n, g.h, g.n_patch = n, h, 0
    p = ndgp._Params()
    p.rc, p.beta, p.a, p.omega_m, p.tol = 1.0, 2.7, 1.0, 0.3, 1e-10
    for k, v in kw.items():
        setattr(p, k, v)
    return g, p


def test_workspace_bytes_and_validation(L):
    g, p = _args()
    nb = L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p))
    # domain level: phi copy + source (2 n^3 doubles) plus the coarser levels
    assert nb >= 2 * 32**3 * 8
    assert nb < 4 * 32**3 * 8
    for n in (12, 4, 2048):
        g, p = _args(n=n)
        assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
        assert b"power of two" in L.ndgp_last_error()
    g, p = _args(h=-1.0)
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
    g, p = _args(beta=0.0)
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
    g, p = _args(max_cycles=5000)
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
    # every documented flag is accepted, any other bit refused
    g, p = _args(flags=ndgp.WARM_START | ndgp.PROFILE | ndgp.TWO_PASS | ndgp.DAMPED)
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) > 0
    g, p = _args(flags=16)
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
    assert b"flag" in L.ndgp_last_error()
    # patch 2 must sit inside patch 1 with margin
    g, p = _args(n=64)
    g.n_patch = 2
    g.patch_n[0], g.patch_n[1] = 64, 32
    g.patch_origin[0][:] = [16, 16, 16]
    g.patch_origin[1][:] = [16, 16, 16]
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) > 0
    g.patch_origin[1][:] = [0, 16, 16]
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
    assert b"patch 2" in L.ndgp_last_error()


def _nested(g, depth, m=32, origin=8):
    """``depth`` patches of m cells, each centred in its parent of m cells."""
    g.n_patch = depth
    for q in range(depth):
        g.patch_n[q] = m
        g.patch_origin[q][:] = [origin] * 3


def test_truncation_level_validation_and_workspace(L):
    """NDGP_MODE_TRUNCATED: trunc_level in [1, n_patch + 1]; only the relaxed
    patches get multigrid hierarchies, so the workspace grows with the level,
    from the interpolated mode's (level 1) to the full mode's (n_patch + 1)."""
    g, p = _args(mode=ndgp.MODE_FULL)
    _nested(g, 4)
    full = L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p))
    p.mode = ndgp.MODE_INTERPOLATED
    interp = L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p))
    assert 0 < interp < full
    p.mode = ndgp.MODE_TRUNCATED
    sizes = []
    for k in range(1, 6):
        p.trunc_level = k
        sizes.append(L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))
    assert sizes[0] == interp and sizes[-1] == full
    assert all(a < b for a, b in zip(sizes, sizes[1:]))
    for k in (0, 6, -1):
        p.trunc_level = k
        assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
        assert b"trunc_level" in L.ndgp_last_error()
    # other modes ignore trunc_level
    p.mode, p.trunc_level = ndgp.MODE_FULL, 99
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == full
    p.mode = 3
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
    # a patch next to its parent's edge fits as an interpolated level (its own
    # cells only) but not as a relaxed one (the 8^3 level's stencil reaches out)
    g, p = _args(mode=ndgp.MODE_TRUNCATED, trunc_level=3)
    _nested(g, 3)
    g.patch_origin[2][:] = [16, 8, 8]
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) > 0
    p.trunc_level = 4
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
    assert b"patch 3" in L.ndgp_last_error()
    # at most NDGP_MAX_PATCHES levels
    g, p = _args()
    g.n_patch = ndgp.MAX_PATCHES + 1
    assert L.ndgp_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0
    with pytest.raises(ValueError):
        ndgp.Grid(n=32, h=1e-3, patches=[ndgp.Patch(32, (8, 8, 8))] * 5)._c()


def test_solve_rejects_bad_arguments_before_gpu_work(L):
    arr = (ctypes.c_void_p * (1 + ndgp.MAX_PATCHES))()
    g, p = _args(n=12)
    st = L.ndgp_solve(ctypes.byref(g), ctypes.byref(p), arr, arr, None, 0, None, None)
    assert st == ndgp.NDGP_EINVAL
    g, p = _args()
    st = L.ndgp_solve(ctypes.byref(g), ctypes.byref(p), arr, arr, None, 0, None, None)
    assert st == ndgp.NDGP_EINVAL  # NULL arrays
    arr[0] = 0x1000  # never dereferenced: the workspace check fails first
    st = L.ndgp_solve(ctypes.byref(g), ctypes.byref(p), arr, arr, None, 0, None, None)
    assert st == ndgp.NDGP_ENOMEM
    assert b"workspace" in L.ndgp_last_error()
