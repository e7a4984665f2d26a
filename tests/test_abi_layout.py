"""The ctypes structures of the Python binding have the layout of the C
structures in include/cae.h: a small C program compiled against the header
prints the size of every structure and the offset of every field, and both
must equal what ctypes computes (CPU only; needs gcc)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


def _layouts():
    from paper_1603_09133_amd import _lib
    return {"cae_options_t": _lib.Options, "cae_stats_t": _lib.Stats, "cae_level_info_t": _lib.LevelInfo,
            "cae_problem_t": _lib.Problem}


def test_ctypes_structures_match_the_header(tmp_path):
    structs = _layouts()
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "cae.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            *key, val = line.split()
            got[tuple(key)] = int(val)
    import ctypes
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
