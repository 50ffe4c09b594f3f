"""The ctypes structures of the Python binding match the C header field by field: a small C
program built against include/hpmocd.h prints each struct's size and every field's offset,
and the binding's ctypes definitions must agree (a mismatch would corrupt values silently)."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2506_01752_amd as hp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# C struct name -> the binding's ctypes class
STRUCTS = {
    "hpmocd_params": hp.Params,
    "hpmocd_front": hp._Front,
    "hpmocd_state_view": hp._View,
    "hpmocd_profile": hp.Profile,
    "hpmocd_snapshot": hp._Snapshot,
    "hpmocd_server_config": hp.ServerConfig,
    "hpmocd_request_info": hp.RequestInfo,
    "hpmocd_server_stats": hp.ServerStats,
}


def c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hpmocd.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        name, key, value = line.split()
        layout[(name, key)] = int(value)
    return layout


def test_ctypes_structs_match_the_header(tmp_path):
    layout = c_layout(tmp_path)
    for name, cls in STRUCTS.items():
        assert ctypes.sizeof(cls) == layout[(name, "size")], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == layout[(name, field)], (name, field)
