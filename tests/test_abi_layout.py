"""The ctypes structures of the binding match include/agis.h byte for byte
(sizes and field offsets as compiled by the C compiler)."""

import ctypes
import os
import subprocess

import pytest

A = pytest.importorskip("paper_2601_01388_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "agis_pattern": A.agis_pattern,
    "agis_plan": A.agis_plan,
    "agis_run_params": A.agis_run_params,
    "agis_result": A.agis_result,
    "agis_tuning": A.agis_tuning,
}


def test_struct_layouts_match_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "agis.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append('printf("agis_record size %zu\\n", sizeof(agis_record));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for name, cls in STRUCTS.items():
        assert int(got[f"{name} size"]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)
    assert int(got["agis_record size"]) == A.RECORD_BYTES
