"""Host-side checks of the C-ABI library (no GPU needed, no compute call made)."""
import ctypes
import os
import re

import pytest

from paper_1502_04025_amd import sapdd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sapdd.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sapdd_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert header_functions() == sorted(sapdd.EXPORTS)


@pytest.mark.skipif(not os.path.exists(sapdd.LIB_PATH), reason="library not built")
def test_library_loads_and_exports_every_header_symbol():
    lib = ctypes.CDLL(sapdd.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name
    sapdd.load_library()


def test_params_struct_matches_header_layout():
    # int block[4], 4 ints, a double, 2 ints -> 48 bytes with natural alignment
    assert ctypes.sizeof(sapdd.Params) == 48
    assert ctypes.sizeof(sapdd.Stats) == 3 * 4 + 4 + 7 * 8


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1502_04025_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", src).replace("oracle's", ""), f
