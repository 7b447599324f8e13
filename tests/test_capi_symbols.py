"""The C-ABI library loads and exports every symbol include/*.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("fh.h", "fh_net.h")]
LIB = os.path.join(ROOT, "paper_2203_02962_amd", "libfh.so")


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fh_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["fh_create", "fh_destroy", "fh_set_grid", "fh_set_phases", "fh_set_load",
              "fh_solve", "fh_get_fluctuation", "fh_get_homogenized"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfh.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfh.so not built")
def test_binding_covers_every_declared_symbol():
    from paper_2203_02962_amd import fh
    assert sorted(fh.EXPORTED) == declared_functions()
    fh.load_library()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2203_02962_amd import fh
    saved = fh._lib
    fh._lib = None
    try:
        with pytest.raises(RuntimeError):
            fh.load_library(str(tmp_path / "missing.so"))
    finally:
        fh._lib = saved
