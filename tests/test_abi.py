"""The C ABI library builds for gfx950, loads, and exports every function include/ipmsk.h declares.

CPU only: no function of the library is called.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipmsk.h")
LIB = os.path.join(ROOT, "paper_2209_08722_amd", "libipmsk.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(ipm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for required in ("ipm_sketch", "ipm_precond_factor", "ipm_pcg_solve", "ipm_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_the_header():
    from paper_2209_08722_amd import native
    bound = {name for name, _, _ in native.SIGNATURES}
    assert set(declared_functions()) <= bound


STRUCTS = {"IpmMatrix": "ipm_matrix", "IpmProblem": "ipm_problem", "IpmState": "ipm_state",
           "IpmParams": "ipm_params", "IpmPcgInfo": "ipm_pcg_info", "IpmStepInfo": "ipm_step_info"}


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the C structs have the size and field offsets the C compiler gives them."""
    import shutil
    import subprocess
    from paper_2209_08722_amd import native
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ipmsk.h"', "int main(void) {"]
    expect = []
    for py, cname in STRUCTS.items():
        cls = getattr(native, py)
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for fname, _ in cls._fields_:
            if fname == "reserved":
                continue
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
            expect.append(getattr(cls, fname).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect


def test_product_path_does_not_import_the_oracle():
    """The binding and the library sources never reference the oracle package."""
    pkg = os.path.join(ROOT, "paper_2209_08722_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text, f
