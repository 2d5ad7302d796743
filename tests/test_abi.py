"""CPU checks of the C boundary: the library builds, loads, and exports exactly
the entry points that include/trbdg.h declares (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trbdg.h")
LIB = os.path.join(ROOT, "paper_2107_07776_amd", "libtrbdg.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"TBDG_API\s+[\w\s\*]+?\b(tbdg_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2107_07776_amd import build
        build.build()
    return LIB


def test_header_declares_entry_points():
    names = declared()
    for n in ("tbdg_create", "tbdg_apply_momentum", "tbdg_apply_pressure", "tbdg_solve_momentum",
              "tbdg_solve_pressure", "tbdg_step", "tbdg_rhs_momentum", "tbdg_rhs_pressure",
              "tbdg_grad_p", "tbdg_diag_momentum", "tbdg_diag_pressure"):
        assert n in names


def test_exports_match_header(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted(set(m for m in re.findall(r"\bT (tbdg_\w+)", out)))
    assert exported == declared()
    from paper_2107_07776_amd import EXPORTED
    assert sorted(EXPORTED) == declared()


def test_library_loads(lib_path):
    lib = ctypes.CDLL(lib_path)
    for n in declared():
        assert getattr(lib, n) is not None


def test_null_arguments_are_rejected_without_a_gpu(lib_path):
    from paper_2107_07776_amd.trbdg import load_library
    lib = load_library(lib_path)
    # every entry point validates its context before touching the device
    assert lib.tbdg_create(None, None, None, None) == -1
    assert lib.tbdg_apply_pressure(None, 1, None, None) == -1
    assert lib.tbdg_step(None, None, None, None, None) == -1
    assert lib.tbdg_last_error(None) == b"null context"


def test_binding_structs_match_header(tmp_path):
    """Every struct the Python binding mirrors has the size and field offsets
    that a C compiler gives the header's declaration."""
    from paper_2107_07776_amd import trbdg as b
    mirrors = {"tbdg_mesh_desc": b.MeshDesc, "tbdg_disc_desc": b.DiscDesc,
               "tbdg_solver_opts": b.SolverOpts, "tbdg_mg_desc": b.MGDesc,
               "tbdg_solve_info": b.SolveInfo, "tbdg_state": b.State}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void) {']
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append('  return 0;\n}')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, key, val = ln.split()
        got[(cname, key)] = int(val)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
