"""The C ABI library builds, loads and exports every declared entry point;
argument checks that run before any HIP call work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helmg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_2308_13476_amd import _binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libhelmg.so not built")
    return B.lib(), B


def test_header_declares_the_expected_entry_points():
    decl = _declared()
    for name in ["mg_setup", "mg_solve", "mg_grad", "mg_destroy", "mg_workspace_bytes", "mg_update_k2"]:
        assert name in decl


def test_library_exports_every_declared_symbol():
    L, B = _lib()
    decl = _declared()
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(B.EXPORTED) == decl


def test_workspace_size_and_argument_checks_without_gpu():
    L, B = _lib()
    opts = B.SetupOpts(B.MG_FP64, 1, 4, 0, None)
    assert L.mg_workspace_bytes(64, 0, B.MG_TRANSFER_BEZIER, ctypes.byref(opts)) > 0
    assert L.mg_workspace_bytes(63, 0, B.MG_TRANSFER_BEZIER, ctypes.byref(opts)) == 0  # not halvable to 4
    assert L.mg_workspace_bytes(64, 9, B.MG_TRANSFER_BEZIER, ctypes.byref(opts)) == 0  # too many levels
    assert L.mg_workspace_bytes(4096, 3, B.MG_TRANSFER_BEZIER, ctypes.byref(opts)) == 0  # coarsest too large
    big = B.SetupOpts(B.MG_FP32_REFINED, 4, 4, 0, None)
    assert L.mg_workspace_bytes(64, 0, 0, ctypes.byref(big)) > L.mg_workspace_bytes(64, 0, 0, ctypes.byref(opts))
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: the checks fail first
    assert L.mg_setup(fake, 64, -1.0, 0.1, 0, 0, ctypes.byref(opts), fake, 1 << 30, None, ctypes.byref(h)) == B.MG_E_ARG
    assert b"h must be" in L.mg_last_error(None)
    assert L.mg_setup(fake, 64, 1 / 64, -0.5, 0, 0, ctypes.byref(opts), fake, 1 << 30, None,
                      ctypes.byref(h)) == B.MG_E_ARG
    assert L.mg_setup(fake, 63, 1 / 63, 0.1, 0, 0, ctypes.byref(opts), fake, 1 << 30, None,
                      ctypes.byref(h)) == B.MG_E_ARG
    assert L.mg_setup(fake, 64, 1 / 64, 0.1, 0, 7, ctypes.byref(opts), fake, 1 << 30, None,
                      ctypes.byref(h)) == B.MG_E_ARG
    small = ctypes.c_size_t(16)
    assert L.mg_setup(fake, 64, 1 / 64, 0.1, 0, 0, ctypes.byref(opts), fake, small, None,
                      ctypes.byref(h)) == B.MG_E_WORKSPACE
    assert L.mg_solve(None, fake, fake, 1, 1e-6, 1, 1, None, None, None) == B.MG_E_ARG
    assert L.mg_status_string(B.MG_E_DIVERGED) == b"MG_E_DIVERGED"


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes struct of the binding has the size and field offsets that a
    C compiler gives the structs of include/helmg.h."""
    import shutil
    import subprocess
    from paper_2308_13476_amd import _binding as B
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    pairs = {"mg_setup_opts": B.SetupOpts, "mg_solve_opts": B.SolveOpts, "mg_solve_stats": B.SolveStats,
             "mg_tune_result": B.TuneResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "helmg.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
