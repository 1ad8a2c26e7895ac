"""CPU checks of the C-ABI library: it is built, loads, and exports every
function declared in include/vie.h (no device calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vie.h")
LIB = os.path.join(ROOT, "paper_1809_05334_amd", "libvie.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vie_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ("vie_mesh_upload", "vie_fill", "vie_precond_factor", "vie_solve", "vie_absorption"):
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libvie.so not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1809_05334_amd import vie
    assert set(declared_functions()) <= set(vie._SIGS)
