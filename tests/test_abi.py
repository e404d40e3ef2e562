"""The C-ABI library loads and exports every function include/ebbkc.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebbkc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ebbkc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ebbkc_prepare", "ebbkc_count", "ebbkc_list", "ebbkc_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2311_13798_amd as ebb
    if not os.path.exists(ebb.LIB_PATH):
        pytest.skip("libebbkc.so not built")
    lib = ctypes.CDLL(ebb.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(ebb.EXPORTED) == set(declared_functions())


def test_strerror_and_defaults_without_gpu():
    import paper_2311_13798_amd as ebb
    if not os.path.exists(ebb.LIB_PATH):
        pytest.skip("libebbkc.so not built")
    assert ebb.ebbkc_strerror(ebb.E_BAD_CSR).startswith("input is not")
    o = ebb.ebbkc_default_options()
    assert (o.early_termination, o.t_plex, o.rule1, o.rule2) == (1, 0, 1, 1)


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2311_13798_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text and "orc_" not in text, f
