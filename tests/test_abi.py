"""The C-ABI library: it builds into the package, loads, and exports every
symbol include/tvs.h declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvs.h")
LIB = os.path.join(ROOT, "paper_2602_17494_amd", "libtvs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tvs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tvs_step1", "tvs_step2", "tvs_schwarz_solve", "tvs_ctx_create",
              "tvs_ctx_destroy", "tvs_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtvs.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtvs.so not built (run __graft_entry__.build())")
def test_binding_mirrors_the_header():
    from paper_2602_17494_amd import tvs
    assert sorted(tvs.EXPORTED) == declared_functions()
    # struct layouts of the binding match the C declarations
    assert ctypes.sizeof(tvs.Params) == 5 * 8 + 8
    assert ctypes.sizeof(tvs.Layout) == 4 * 4 + 8
    assert ctypes.sizeof(tvs.Iters) == 8 + 8
    assert ctypes.sizeof(tvs.Stats) == 8 + 4 * 8


def test_binding_refuses_to_run_without_library(monkeypatch, tmp_path):
    from paper_2602_17494_amd import tvs
    monkeypatch.setattr(tvs, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(tvs, "_lib", None)
    with pytest.raises(RuntimeError):
        tvs.load()
