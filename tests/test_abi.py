"""The C-ABI library loads on the CPU host and exports every function include/sg.h declares.
No compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2209_14740_amd", "libsg.so")


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(sg_[a-z0-9_]+)\s*\(", src))
    return sorted(n for n in names if not n.endswith("_cb"))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("sg_setup", "sg_apply", "sg_precond", "sg_gmres", "sg_fgmres"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsg.so not built")
def test_strerror_without_gpu():
    from paper_2209_14740_amd import sg
    L = sg.lib()
    assert L.sg_strerror(0) == b"ok"
    assert b"invalid" in L.sg_strerror(-1)
    assert L.sg_strerror(-99) == b"unknown status"


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_2209_14740_amd import sg
    monkeypatch.setattr(sg, "_lib", None)
    monkeypatch.setattr(sg, "_LIB_PATH", "/nonexistent/libsg.so")
    with pytest.raises(ImportError):
        sg.lib()
