"""The C-ABI library loads and exports every function include/*.h declares
(no compute calls: no GPU is needed)."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(pic_\w+)\s*\(", src, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("pic_create", "pic_fields_load", "pic_push_subcycled", "pic_diag"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2102_10983_amd import picsub
    if not os.path.exists(picsub.LIB_PATH):
        pytest.fail("libpicsub.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(picsub.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(picsub.EXPORTS) == set(_declared())


def test_binding_declares_signatures_without_gpu():
    from paper_2102_10983_amd import picsub
    L = picsub.load_library()
    assert L.pic_push_subcycled.argtypes is not None
    assert L.pic_last_error(None) == b"null context"
    assert L.pic_destroy(None) == 1      # PIC_E_ARG, no GPU touched


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2102_10983_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*.*"), recursive=True):
        if path.endswith((".py", ".hip", ".h", ".cpp")):
            text = open(path).read()
            assert not re.search(r"^\s*(from|import)\s+oracle\b", text, re.M), path
            assert "liboracle" not in text and "orc_" not in text, path
