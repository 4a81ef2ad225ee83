"""The Python binding's ctypes structures against the C layout of
include/spamm.h: a small C program compiled here with gcc prints the size of
every public struct and the offset of every field, which must equal what
ctypes computes for the binding's classes (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

import paper_1203_1692_amd as sp
from paper_1203_1692_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "spamm_opts": _binding.Opts,
    "spamm_stats": _binding.Stats,
    "spamm_request": _binding.Request,
    "spamm_result": _binding.Result,
    "spamm_server_stats": _binding.ServerStats,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "spamm.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    table = {}
    for line in out.splitlines():
        s, f, v = line.split()
        table[(s, f)] = int(v)
    return table


@pytest.mark.parametrize("cname", list(STRUCTS))
def test_struct_size_and_offsets_match(c_layout, cname):
    import ctypes
    cls = STRUCTS[cname]
    assert ctypes.sizeof(cls) == c_layout[(cname, "size")], cname
    for fname, _ in cls._fields_:
        assert getattr(cls, fname).offset == c_layout[(cname, fname)], (cname, fname)


def test_every_header_struct_field_is_bound():
    """Each field declared in the header's public structs has a ctypes field."""
    import re
    text = open(sp.HEADER).read()
    for cname, cls in STRUCTS.items():
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = re.findall(r"\b(\w+)\s*(?:\[[^\]]*\])?\s*;", body)
        bound = {f for f, _ in cls._fields_}
        assert set(names) == bound, (cname, set(names) ^ bound)
