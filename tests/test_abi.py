"""CPU-side checks of the boundary: the library builds, loads, and exports every symbol the
public header declares; header and binding agree.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hopf.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hopf_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    from paper_1605_01799_amd import _lib
    assert header_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_1605_01799_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhopf.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name
    lib = _lib.load()
    assert b"gfx950" in lib.hopf_version()


def test_descriptor_layout_matches_header():
    """The ctypes descriptor mirrors hopf_problem_desc field by field (C layout rules)."""
    from paper_1605_01799_amd import _lib
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} hopf_problem_desc;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b(\w+)\s*;", body)
    py = [f[0] for f in _lib.ProblemDesc._fields_]
    assert [n if n != "lambda" else "lam" for n in names] == py


def test_oracle_is_not_imported_by_product_code():
    """The product path never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1605_01799_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", src).lower() or f == "workloads.py", f


def test_deterministic_setting():
    """hopf_set_deterministic: a process-wide flag that takes 0 or 1 (no device call is made)."""
    from paper_1605_01799_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhopf.so not built")
    lib = _lib.load()
    assert lib.hopf_get_deterministic() == 0
    try:
        assert lib.hopf_set_deterministic(1) == _lib.HOPF_OK
        assert lib.hopf_get_deterministic() == 1
        assert lib.hopf_set_deterministic(2) == _lib.HOPF_EINVAL
        assert b"0 or 1" in lib.hopf_last_error()
        assert lib.hopf_get_deterministic() == 1  # unchanged on error
    finally:
        assert lib.hopf_set_deterministic(0) == _lib.HOPF_OK
    assert lib.hopf_get_deterministic() == 0
