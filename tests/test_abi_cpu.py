"""Host-side checks of the C-ABI library: it is built, loads, and exports
every entry point declared in include/sgo.h.  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgo.h")
LIB = os.path.join(ROOT, "paper_1603_02732_amd", "libsgo.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sgo_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1603_02732_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ["sgo_create", "sgo_set_cell", "sgo_set_atoms", "sgo_set_cutoff", "sgo_scf",
                 "sgo_energy", "sgo_forces", "sgo_batch_scf"]:
        assert need in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_exports_are_plain_c(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (sgo_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_version_and_null_handles(lib):
    lib.sgo_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.sgo_version()
    # NULL handles are rejected without touching a device
    assert lib.sgo_destroy(None) == -1
    assert lib.sgo_scf(None, None, None) == -1
    assert lib.sgo_batch_destroy(None) == -1
    lib.sgo_last_error.restype = ctypes.c_char_p
    lib.sgo_last_error(None)


def test_binding_signatures_cover_header():
    import paper_1603_02732_amd as pkg
    lib = pkg.load_library()
    for n in declared_functions():
        assert getattr(lib, n).argtypes is not None or n in ("sgo_version",), n
