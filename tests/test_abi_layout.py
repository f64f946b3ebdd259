"""The ctypes mirrors of the C ABI's structs match include/pamd.h field by
field: a small C program compiled against the header prints sizeof and every
offsetof, and they are compared with the binding's Structure classes.  A
mismatch would make the library read arguments at the wrong offsets without
any error, so this runs on the host with no device."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1907_09529_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "pamd_potential": _lib.PamdPotential,
    "pamd_path": _lib.PamdPath,
    "pamd_tuning": _lib.PamdTuning,
    "pamd_launch": _lib.PamdLaunch,
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_struct_layouts_match_header(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pamd.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    c_side = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        c_side[(cname, field)] = int(value)
    for cname, py in STRUCTS.items():
        assert c_side[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert c_side[(cname, field)] == getattr(py, field).offset, (cname, field)


def test_every_c_field_is_mirrored():
    # the header's field names of each struct, in order, equal the binding's
    text = open(os.path.join(ROOT, "include", "pamd.h")).read()
    for cname, py in STRUCTS.items():
        body = text[text.index(f"typedef struct {cname} {{"):]
        body = body[body.index("{") + 1:body.index(f"}} {cname};")]
        names = []
        for decl in body.split(";"):
            decl = decl.split("*/")[-1].strip()
            if decl and not decl.startswith("/*"):
                names.append(decl.split()[-1])
        assert names == [f for f, _ in py._fields_], cname
