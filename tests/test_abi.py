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
    assert (o.early_termination, o.t_plex, o.rule1, o.rule2, o.ordering) == (1, 0, 1, 1, 0)


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors of the option / info / result structs have the C sizes and offsets
    import ctypes
    import subprocess
    import paper_2311_13798_amd as ebb
    src = tmp_path / "sizes.c"
    src.write_text('''#include <stddef.h>
#include <stdio.h>
#include "ebbkc.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu\\n", sizeof(ebbkc_options), offsetof(ebbkc_options, ordering),
           offsetof(ebbkc_options, dense_k4), sizeof(ebbkc_info), offsetof(ebbkc_info, prepare_ms));
    return 0;
}
''')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    O, I = ebb.ebbkc_options, ebb.ebbkc_info
    assert got == [ctypes.sizeof(O), O.ordering.offset, O.dense_k4.offset, ctypes.sizeof(I), I.prepare_ms.offset]


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2311_13798_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text and "orc_" not in text, f
