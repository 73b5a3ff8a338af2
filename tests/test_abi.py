"""The C-ABI library loads and exports every function include/dpmi.h
declares (CPU only: no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dpmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("dp_create", "dp_set_model", "dp_compute", "dp_md_run", "dp_destroy", "dp_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2005_00223_amd import _lib
    L = _lib.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_lib.EXPORTS) == set(_declared())


def test_exports_are_c_symbols():
    from paper_2005_00223_amd import _lib
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    syms = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for n in _declared():
        assert n in syms, n


def test_null_context_errors_without_gpu():
    from paper_2005_00223_amd import _lib
    L = _lib.lib()
    assert L.dp_last_error(None) == b"NULL context"
    assert L.dp_compute(None, 0, None, None, None, None, None, None) == _lib.DP_E_ARG
    assert L.dp_set_model(None, b"", 0, 0) == _lib.DP_E_ARG
    L.dp_destroy(None)


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes mirrors of the structs in include/dpmi.h have the
    C layout (size and every field offset), checked with the host compiler."""
    import subprocess
    from paper_2005_00223_amd import _lib
    structs = {"dp_stats": _lib.dp_stats, "dp_student_cfg": _lib.dp_student_cfg}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "dpmi.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
