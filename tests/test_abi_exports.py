"""The C-ABI library loads without a GPU and exports every declared function."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2203_14906_amd", "libhodmas.so")


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        names += re.findall(r"\b(hodmas_\w+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("hodmas_plan", "hodmas_beamform", "hodmas_destroy", "hodmas_status_string"):
        assert core in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version():
    from paper_2203_14906_amd import hodmas
    assert hodmas.status_string(0) == "ok"
    assert hodmas.status_string(1) == "invalid argument"
    assert hodmas.status_string(99) == "unknown status"
    assert "gfx950" in hodmas.version()
