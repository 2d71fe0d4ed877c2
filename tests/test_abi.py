"""The C-ABI library loads without a GPU and exports every declared symbol."""
import os
import re

from paper_2506_06494_amd import jgs2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "jgs2.h")).read()
    return sorted(set(re.findall(r"\b(jgs2_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared() == sorted(jgs2.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = jgs2.load()
    for name in declared():
        assert hasattr(lib, name), name


def test_index_checked_library_exports_the_same_symbols():
    """libjgs2_bounds.so (the same sources with JGS2_BOUNDS_CHECK) is a drop-in
    twin of libjgs2.so: it loads without a GPU and exports every declared
    symbol.  Skipped when it has not been built."""
    import ctypes
    import pytest
    if not os.path.exists(jgs2.BOUNDS_LIB_PATH):
        pytest.skip("libjgs2_bounds.so is not built")
    lib = ctypes.CDLL(jgs2.BOUNDS_LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name


def test_default_params():
    p = jgs2.default_params()
    assert abs(p.dt - 1 / 120) < 1e-15 and p.gravity[1] == -9.8 and p.check_every == 8
