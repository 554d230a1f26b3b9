"""The ctypes mirrors of the C-ABI structs in include/smpm_schur.h: every
field at the offset and of the size the C compiler gives it, and the same
total size, so a field added on one side only fails here instead of shifting
what the library writes."""
import ctypes
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_1512_01756_amd as P  # noqa: E402

MIRRORS = [("smpm_grid", P.Grid), ("smpm_opts", P.Opts), ("smpm_stats", P.Stats), ("smpm_info", P.Info)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a C compiler")
def test_struct_layouts_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "smpm_schur.h"', "int main(void) {"]
    for cname, cls in MIRRORS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu %zu\\n", offsetof({cname}, {fname}), '
                         f"sizeof((({cname} *)0)->{fname}));")
    lines += ["  return 0;", "}"]
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    c = {}
    for ln in out:
        f = ln.split()
        if len(f) == 3:
            c[(f[0], "")] = (int(f[2]),)
        elif len(f) == 4:
            c[(f[0], f[1])] = (int(f[2]), int(f[3]))
    for cname, cls in MIRRORS:
        assert c[(cname, "")] == (ctypes.sizeof(cls),), cname
        for fname, ftype in cls._fields_:
            assert c[(cname, fname)] == (getattr(cls, fname).offset, ctypes.sizeof(ftype)), (cname, fname)
