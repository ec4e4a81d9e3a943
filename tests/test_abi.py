"""CPU-side checks of the C-ABI library: it loads, and it exports every
function that include/chl.h declares. No device work is started here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "chl.h")
LIB = os.path.join(ROOT, "paper_1907_00140_amd", "libchl.so")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(chl_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_1907_00140_amd.build as b
        b.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_parses():
    names = declared()
    for must in ("chl_build", "chl_query", "chl_labels_export", "chl_labels_free",
                 "chl_error_string", "chl_build_stats", "chl_server_create"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_strings(lib):
    f = lib.chl_error_string
    f.restype = ctypes.c_char_p
    f.argtypes = [ctypes.c_int]
    seen = set()
    for code in range(0, -7, -1):
        s = f(code)
        assert s and s not in seen
        seen.add(s)
    assert f(-99) == b"unknown error"


def test_binding_signatures_cover_header():
    from paper_1907_00140_amd import chl
    lib = chl.load()
    for n in declared():
        assert getattr(lib, n).argtypes is not None or n == "chl_error_string", n


def test_product_does_not_reach_the_oracle():
    """The product package never imports the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1907_00140_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "chl_oracle" not in txt, f


def test_build_entry_resolves_the_build_module():
    """__graft_entry__.build() compiles through paper_1907_00140_amd.build:
    the package must not shadow that submodule with another object."""
    import importlib
    import types
    import paper_1907_00140_amd as pkg
    assert not callable(getattr(pkg, "build", None)) or isinstance(pkg.build, types.ModuleType)
    b = importlib.import_module("paper_1907_00140_amd.build")
    assert callable(b.build)
    import __graft_entry__ as ge
    assert callable(ge.build) and callable(ge.smoke)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's field
    offsets and sizes (a field added on one side only would shift every
    later one)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    from paper_1907_00140_amd import chl
    mirrors = {"chl_graph": chl.CGraph, "chl_allocator": chl.CAllocator, "chl_build_opts": chl.CBuildOpts,
               "chl_stats": chl.CStats, "chl_server_opts": chl.CServerOpts}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "chl.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, cls in mirrors.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
