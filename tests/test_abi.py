"""The C-ABI library loads and exports every entry point the header declares
(no compute calls).  The checks run on the CPU when the library is built here,
and again, marked gpu, on the GPU machine, where the built library must exist."""
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


def _exports():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.cavdftb_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.cavdftb_version()


def _binding():
    from paper_2512_03277_amd.binding import SYMBOLS
    assert sorted(SYMBOLS) == declared()


def _invalid_arguments():
    lib = ctypes.CDLL(LIB)
    lib.cavdftb_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.cavdftb_create(None, None, None, ctypes.byref(out)) == -1
    assert lib.cavdftb_destroy(None) == -1
    assert lib.cavdftb_eval_units(None, None, None, None, None, None, None) == -1


CHECKS = [_exports, _binding, _invalid_arguments]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_library_abi_on_cpu(check):
    check()


@pytest.mark.gpu
@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_library_abi_on_gpu_box(check):
    assert os.path.exists(LIB), "libcavdftb.so is not built"
    check()
