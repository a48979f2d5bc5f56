"""The C-ABI library loads and exports every symbol that include/hg.h declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hg.h")
LIB = os.path.join(ROOT, "paper_2609_07577_amd", "libhgcoarsen.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2609_07577_amd import build
        build.build()
    return LIB


def test_header_declares_the_three_operations():
    syms = declared_symbols()
    for s in ("hg_coarsen_level", "hg_contract", "hg_connectivity"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_exported_list_matches_binding(lib_path):
    from paper_2609_07577_amd import hg
    assert sorted(hg.EXPORTED) == declared_symbols()


def test_symbols_are_c_linkage(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True,
                         text=True).stdout
    names = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for s in declared_symbols():
        assert s in names, f"{s} is not an unmangled export"


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "hg.h"\nint main(void){hg_limits l={1,2,3};(void)l;return 0;}\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", f"-I{os.path.dirname(HEADER)}",
                        str(src), "-c", "-o", str(tmp_path / "t.o")], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr
