"""Host-side checks of the C-ABI library (no GPU needed, no compute call made)."""
import ctypes
import os
import re
import subprocess

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


def test_params_struct_matches_header_layout(tmp_path):
    """The ctypes mirrors have the size and field offsets the C compiler gives the header's
    structs."""
    fields_p = [f for f, _ in sapdd.Params._fields_]
    fields_s = [f for f, _ in sapdd.Stats._fields_]
    fields_m = [f for f, _ in sapdd.MgParams._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"sapdd.h\"\nint main(void) {\n"
                   + f'  printf("%zu %zu %zu\\n", sizeof(sapdd_params), sizeof(sapdd_stats), sizeof(sapdd_mg_params));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(sapdd_params, {f}));\n' for f in fields_p)
                   + "".join(f'  printf("%zu\\n", offsetof(sapdd_stats, {f}));\n' for f in fields_s)
                   + "".join(f'  printf("%zu\\n", offsetof(sapdd_mg_params, {f}));\n' for f in fields_m)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(sapdd.Params)
    assert int(out[1]) == ctypes.sizeof(sapdd.Stats)
    assert int(out[2]) == ctypes.sizeof(sapdd.MgParams)
    offs = [int(v) for v in out[3:]]
    n_p, n_s = len(fields_p), len(fields_s)
    assert offs[:n_p] == [getattr(sapdd.Params, f).offset for f in fields_p]
    assert offs[n_p:n_p + n_s] == [getattr(sapdd.Stats, f).offset for f in fields_s]
    assert offs[n_p + n_s:] == [getattr(sapdd.MgParams, f).offset for f in fields_m]


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1502_04025_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", src).replace("oracle's", ""), f


def test_fp16_site_scale_rule_on_the_host(tmp_path):
    """The FP16 storage helpers' scale reciprocal (core.hpp fp16_site_inv), compiled for the
    host: finite for every finite maximum, zero for a maximum below the smallest normal
    float (such a site stores zeros instead of NaN = 0 * inf), and |v| * inv <= 1."""
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "fp16chk"
    subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-Wno-unused-command-line-argument",
                    "-I", os.path.join(ROOT, "paper_1502_04025_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "fp16_scale_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "BAD" not in r.stdout and r.stdout.count(" ok") == 12

