"""CPU test: the binding's ctypes structures have the layout of the C
header's structures - the same size and the same offset for every field -
read from a small C program compiled against include/mpld.h with gcc.  A
field added to one side only would otherwise surface as a struct_size error
(or a silently misread field) on the GPU."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _structs():
    from paper_2303_14335_amd import _ffi
    out = []
    for name in dir(_ffi):
        obj = getattr(_ffi, name)
        if isinstance(obj, type) and issubclass(obj, ctypes.Structure) and name.startswith("mpld_"):
            out.append((name, obj))
    return out


def test_ctypes_structures_match_the_header(tmp_path):
    structs = _structs()
    assert len(structs) >= 10
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mpld.h"', "int main(void) {"]
    for name, cls in structs:
        lines.append(f'  printf("{name} .sizeof %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("the layout probe does not compile against mpld.h:\n" + r.stderr[-2000:])
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for name, cls in structs:
        assert got[(name, ".sizeof")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
