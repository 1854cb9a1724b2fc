"""The ctypes structures of the binding have the layout of the C header:
a C program built with gcc from include/fz.h prints every field's offset and
every structure's size, and each must equal the binding's."""
import ctypes
import os
import subprocess

import pytest

import paper_2405_07989_amd as fz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "fz_query": fz.fz_query,
    "fz_result": fz.fz_result,
    "fz_stats": fz.fz_stats,
    "fz_slice_info": fz.fz_slice_info,
    "fz_tune_result": fz.fz_tune_result,
    "fz_server_cfg": fz.fz_server_cfg,
    "fz_server_stats": fz.fz_server_stats,
}


def test_struct_layouts_match_the_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fz.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                        str(exe)], capture_output=True, text=True)
    if r.returncode:
        pytest.fail("the header does not compile as C: " + r.stderr)
    got = dict(line.rsplit(" ", 1) for line in
               subprocess.run([str(exe)], capture_output=True, text=True, check=True)
               .stdout.splitlines())
    for name, cls in STRUCTS.items():
        assert int(got[f"{name} size"]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"
