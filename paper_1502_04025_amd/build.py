"""Build libsapdd.so (HIP, gfx950) in-tree.

    python -m paper_1502_04025_amd.build          # compile every csrc/*.hip and link
    python -m paper_1502_04025_amd.build --changed  # recompile only sources newer than their object

Each translation unit is compiled separately with hipcc for gfx950 and linked into
paper_1502_04025_amd/libsapdd.so next to this file. Packed-FP32 instructions are switched
off for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsapdd.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD, src[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _deps(path: str, seen=None) -> set:
    """path and the package headers it includes, recursively (quoted includes only)."""
    import re
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    for name in re.findall(r'#include\s+"([^"]+)"', open(path).read()):
        _deps(os.path.normpath(os.path.join(os.path.dirname(path), name)), seen)
    return seen


def _stale(src: str) -> bool:
    """True if the object of src is missing or older than src or a header it includes."""
    obj = os.path.join(BUILD, src[:-4] + ".o")
    if not os.path.exists(obj):
        return True
    return max(os.path.getmtime(d) for d in _deps(os.path.join(CSRC, src))) > os.path.getmtime(obj)


def build(verbose: bool = False, extra=(), only_changed: bool = False) -> str:
    """Compile all sources (only the stale ones with only_changed) and link the shared
    library; returns its path."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = [s for s in srcs if _stale(s)] if only_changed else srcs
    workers = max(1, min(len(todo), 8, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda s: _compile(s, list(extra)), todo))
    objs = [os.path.join(BUILD, s[:-4] + ".o") for s in srcs]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", flush=True)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    changed = "--changed" in args
    build(verbose=True, extra=[a for a in args if a != "--changed"], only_changed=changed)
