"""The C-ABI library loads and exports every symbol include/apx.h declares.

CPU-only: no compute call is made (there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apx.h")
LIB = os.path.join(ROOT, "paper_0910_1650_amd", "libapx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:apx_status|void|char|size_t|int)\s*\*?\s*(\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for want in ("ap_similarity", "ap_iterate", "ap_solve", "ap_solve_batched", "pap_solve", "lap_solve",
                 "apx_create", "apx_destroy"):
        assert want in names, want


@pytest.mark.skipif(not os.path.exists(LIB), reason="libapx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libapx.so not built")
def test_binding_signatures_cover_header():
    import paper_0910_1650_amd as apx
    assert sorted(apx.SIGNATURES) == declared_functions()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_0910_1650_amd as apx
    monkeypatch.setattr(apx, "_lib", None)
    monkeypatch.setattr(apx, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        apx.lib()
