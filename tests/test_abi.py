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
    for required in ("pic_create", "pic_destroy", "pic_last_error", "pic_particles_set",
                     "pic_fields_load", "pic_fields_load_lattice", "pic_push_subcycled",
                     "pic_diag", "pic_batch_create", "pic_fields_load_r", "pic_diag_r",
                     "pic_advance", "pic_predictor_set", "pic_mlp_forward", "pic_mlp_grad",
                     "pic_mlp_adam", "pic_state_export", "pic_state_import", "pic_strict_set"):
        assert required in names, required


def test_header_constants():
    """Status codes (PIC_E_NUMERIC for strict mode), the k_max limit of 12
    and the no-allocation entry point's particle limit."""
    src = open(os.path.join(ROOT, "include", "picsub.h")).read()
    codes = dict(re.findall(r"(PIC_\w+)\s*=\s*(\d+)", src))
    assert [codes[c] for c in ("PIC_OK", "PIC_E_ARG", "PIC_E_DEVICE", "PIC_E_NOMEM",
                               "PIC_E_LEVEL", "PIC_E_STATE", "PIC_E_NUMERIC")] == list("0123456")
    assert re.search(r"#define PIC_K_MAX_LIMIT 12\b", src)
    assert re.search(r"#define PIC_DIAG_NOALLOC_MAX_NP 1572864\b", src)
    from paper_2102_10983_amd import picsub
    assert picsub.STATUS[6] == "PIC_E_NUMERIC"


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
