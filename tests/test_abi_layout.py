"""The ctypes mirrors of the public structs match the C header: a small C
program compiled against include/mpk.h prints sizeof and offsetof of every
field, compared with ctypes (no GPU, no library call)."""
import os
import shutil
import subprocess

import pytest

from paper_2205_01598_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [_lib.mpk_csr, _lib.mpk_options, _lib.mpk_plan_info, _lib.mpk_recurrence]


def test_struct_layout_matches_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "mpk.h"', "int main(void) {"]
    for cls in STRUCTS:
        name = cls.__name__
        lines.append(f'  printf("{name} @sizeof %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.run([cc, "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cls in STRUCTS:
        name = cls.__name__
        assert got[(name, "@sizeof")] == __import__("ctypes").sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
