"""The C-ABI library loads and exports every entry point its header
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qoz.h")
LIB = os.path.join(ROOT, "paper_2310_14133_amd", "libqoz.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qoz_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("qoz_compress", "qoz_decompress", "qoz_tune", "qoz_metrics",
              "qoz_inspect", "qoz_compress_bound", "qoz_ctx_create",
              "qoz_ctx_destroy", "qoz_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libqoz.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_2310_14133_amd as q
    for n in declared():
        assert hasattr(q, n), n


def test_binding_fails_loudly_without_library(monkeypatch):
    import paper_2310_14133_amd as q
    monkeypatch.setattr(q, "_lib", None)
    monkeypatch.setattr(q, "LIB_PATH", "/nonexistent/libqoz.so")
    with pytest.raises(RuntimeError):
        q.lib()


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2310_14133_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                for bad in ("import oracle", "from oracle", "qoz_ref",
                            "libqoz_ref"):
                    assert bad not in src, (f, bad)
