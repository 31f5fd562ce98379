"""The ctypes mirrors of the C structs in paper_2606_28608_amd/pdmk.py against
include/pdmk.h: a small C program built with the host compiler prints the
size of each struct and the offset of every field the binding names; the
binding must agree field by field (a field added to one side only would
shift every later field without an error)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2606_28608_amd import pdmk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "pdmk_opts": pdmk.Opts,
    "pdmk_geometry": pdmk.Geometry,
    "pdmk_stats": pdmk.Stats,
    "pdmk_kernel_info": pdmk.KernelInfo,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    d = tmp_path_factory.mktemp("layout")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pdmk.h"',
             "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));'
                         % (cname, fname, cname, fname))
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        s, f, v = line.split()
        table[(s, f)] = int(v)
    return table


@pytest.mark.parametrize("cname", list(STRUCTS))
def test_struct_matches_header(c_layout, cname):
    cls = STRUCTS[cname]
    assert ctypes.sizeof(cls) == c_layout[(cname, "size")], cname
    for fname, _ in cls._fields_:
        assert getattr(cls, fname).offset == c_layout[(cname, fname)], (cname, fname)
