"""The C-ABI library loads and exports every entry point the header declares
(CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cavdftb.h")
LIB = os.path.join(ROOT, "paper_2512_03277_amd", "libcavdftb.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(cavdftb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_hot_path_calls():
    names = declared()
    for n in ("cavdftb_eval_units", "cavdftb_born_charges", "cavdftb_cavity_forces", "cavdftb_step"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.cavdftb_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.cavdftb_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_the_header():
    from paper_2512_03277_amd.binding import SYMBOLS
    assert sorted(SYMBOLS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_arguments_rejected_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.cavdftb_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.cavdftb_create(None, None, None, ctypes.byref(out)) == -1
    assert lib.cavdftb_destroy(None) == -1
    assert lib.cavdftb_eval_units(None, None, None, None, None, None, None) == -1
