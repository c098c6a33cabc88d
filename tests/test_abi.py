"""The C-ABI library loads and exports every function include/alphacirc.h declares
(no GPU needed: nothing is called that touches a device)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "alphacirc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ac_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2506_03947_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2506_03947_amd import build
        build.build(verbose=False)
    return _lib.LIB_PATH


def test_header_declarations_present():
    names = declared_functions()
    assert "ac_solve" in names and "ac_apply_prec" in names and "ac_apply_A" in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ac_[A-Za-z0-9_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_binding_covers_the_header(lib_path):
    from paper_2506_03947_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)
    _lib.load()


def test_status_strings_without_device(lib_path):
    from paper_2506_03947_amd import _lib
    lib = _lib.load()
    assert lib.ac_status_string(_lib.AC_ERR_ALPHA).decode().startswith("alpha")
    assert lib.ac_status_string(12345).decode() == "unknown status"
