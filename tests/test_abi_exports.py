"""The built library loads and exports every function the public header
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(mrpop_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_three_hot_path_calls():
    names = _declared()
    for n in ("mrpop_fk_spheres", "mrpop_validate_edges"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2609_30644_amd as M
    lib = ctypes.CDLL(M.lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_error_without_device():
    import paper_2609_30644_amd as M
    lib = M.load_library()
    assert b"gfx950" in lib.mrpop_version()
    assert lib.mrpop_last_error(None) is not None


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2609_30644_amd._binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "_HERE", str(tmp_path))
    with pytest.raises(ImportError):
        B.load_library()
