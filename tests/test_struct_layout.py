"""The binding's ctypes structures match the C header field by field: a small
C program built with gcc against include/pa.h prints every struct's size and
each field's offset, and the test compares them with the ctypes layouts."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1609_00061_amd import pa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("pa_axis", pa.Axis), ("pa_relation", pa.Relation), ("pa_bitarray", pa.BitArray),
         ("pa_system", pa.System), ("pa_opts", pa.Opts), ("pa_tuning", pa.Tuning), ("pa_report", pa.Report)]


def _c_layout(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pa.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_ctypes_structs_match_header(tmp_path):
    c = _c_layout(tmp_path)
    for cname, cls in PAIRS:
        assert c[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert c[(cname, field)] == getattr(cls, field).offset, (cname, field)
