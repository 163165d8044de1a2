"""Host-only checks of the device library: it loads, and it exports every entry
point include/mps.h declares (no device calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mps.h")
LIB = os.path.join(ROOT, "paper_1111_3124_amd", "libmps_hip.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mps_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_paper_entry_points():
    names = declared()
    for n in ["mps_create", "mps_apply_gate", "mps_schmidt", "mps_amplitude"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="device library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="device library not built")
def test_binding_mirrors_every_declared_symbol():
    from paper_1111_3124_amd import binding
    for n in declared():
        assert hasattr(binding, n), n
        assert n in binding.EXPORTED
    assert "gfx950" in binding.mps_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="device library not built")
def test_library_is_built_for_gfx950_only():
    data = open(LIB, "rb").read()
    assert b"gfx950" in data
    for other in (b"gfx942", b"gfx90a", b"sm_"):
        assert b"amdgcn-amd-amdhsa--" + other not in data
