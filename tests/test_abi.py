"""The C-ABI library loads and exports every entry point include/hra.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hra.h")
LIB = os.path.join(ROOT, "paper_2609_05467_amd", "libhra.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hra_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for n in ["hra_build_bvh", "hra_sample_surface", "hra_cast_hemisphere", "hra_dominant_axes", "hra_classify",
              "hra_min_setups"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhra.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert ctypes.CDLL(LIB).hra_version  # callable without a device


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhra.so not built")
def test_binding_covers_header():
    from paper_2609_05467_amd import hra
    assert set(declared()) <= set(hra.EXPORTS)
