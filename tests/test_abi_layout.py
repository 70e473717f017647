"""The binding's ctypes structures have the layout of include/ip.h's C
structures: sizes and every field offset, read from a small C program that
includes the header (host compiler only, no GPU)."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = ("ip_fparams", "ip_space", "ip_scene", "ip_stats", "ip_request", "ip_result", "ip_batch_summary")


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    from paper_2406_04795_amd import ip
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "ip.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for name, _ in getattr(ip, s)._fields_:
            lines.append(f'  printf("{s} {name} %zu\\n", offsetof({s}, {name}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("layout")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, name, v = line.split()
        got[(s, name)] = int(v)
    return got


@pytest.mark.parametrize("name", STRUCTS)
def test_struct_layout_matches_header(c_layout, name):
    from paper_2406_04795_amd import ip
    st = getattr(ip, name)
    assert ctypes.sizeof(st) == c_layout[(name, "size")]
    for field, _ in st._fields_:
        assert getattr(st, field).offset == c_layout[(name, field)], field
