"""The C-ABI library loads and exports every entry point include/wilson.h declares
(no device calls: these run without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "wilson.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(wilson_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_two_plain_calls():
    names = declared_functions()
    assert "wilson_dslash" in names and "wilson_solve" in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    from paper_1811_00893_amd import _lib

    lib = _lib.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_host_only_calls():
    from paper_1811_00893_amd import _lib

    assert "gfx950" in _lib.wilson_version()
    assert _lib.wilson_strerror(_lib.WILSON_INVALID_ARG) == "invalid argument"
    assert _lib.wilson_strerror(_lib.WILSON_OK) == "ok"
    # footprint is pure host arithmetic; odd extents are rejected with 0
    assert _lib.wilson_footprint_bytes((8, 8, 8, 8), 1) > 0
    assert _lib.wilson_footprint_bytes((8, 8, 8, 7), 1) == 0
    fp32 = _lib.wilson_footprint_bytes((8, 8, 8, 8), 1, {"precision": _lib.WILSON_FP32})
    fp64 = _lib.wilson_footprint_bytes((8, 8, 8, 8), 1)
    # mixed FP32: 7 FP64 fields + 9 FP32 fields; plain FP64: 12 FP64 fields (plus small buffers)
    assert abs(fp32 / fp64 - 11.5 / 12) < 0.02
    assert _lib.wilson_footprint_bytes((8, 8, 8, 8), 12) > 11 * fp64


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of wilson_solve_opts and wilson_solve_info have the header's size
    and field offsets (a C probe compiled against include/wilson.h prints them)."""
    import ctypes
    import shutil
    import subprocess

    from paper_1811_00893_amd import _lib

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "wilson.h"', "int main(void) {"]
    for st in (_lib.wilson_solve_opts, _lib.wilson_solve_info):
        name = st.__name__
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st in (_lib.wilson_solve_opts, _lib.wilson_solve_info):
        name = st.__name__
        assert got[(name, "size")] == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert got[(name, f)] == getattr(st, f).offset, (name, f)
