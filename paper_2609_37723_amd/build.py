"""Build the HIP library libnucleon.so for gfx950 (in-tree, next to this file).

Each csrc/*.hip file is compiled to an object in parallel (every kernel is
launched from the file that defines it, so no relocatable device code is
needed), then the objects are linked into one shared library.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnucleon.so")
OBJDIR = os.path.join(HERE, "_build")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 VALU ops stay off: the compiler would otherwise emit them from
    # ordinary float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


# Host-only sanitizer builds (the device code is compiled as usual): ASan + UBSan, or TSan.
# Each -fsanitize flag goes to the host pass only. The result is a separate library under
# _build/ that the binding loads when NUC_LIBRARY names it; the sanitizer runtime must be
# preloaded into the process (see sanitize.py).
SANITIZE_FLAGS = {
    "address": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"],
    "thread": ["-Xarch_host", "-fsanitize=thread"],
}


def _compile(src: str, verbose: bool, objdir: str = OBJDIR, extra=()) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = ["hipcc"] + HIP_FLAGS + list(extra) + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False, sanitize: str | None = None) -> str:
    """Compile every csrc/*.hip for gfx950 and link libnucleon.so next to this file, or,
    with sanitize = "address" / "thread", _build/libnucleon_<sanitize>.so."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    extra = SANITIZE_FLAGS[sanitize] if sanitize else []
    objdir = os.path.join(OBJDIR, sanitize) if sanitize else OBJDIR
    lib = os.path.join(OBJDIR, "libnucleon_%s.so" % sanitize) if sanitize else LIB
    os.makedirs(objdir, exist_ok=True)
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, objdir, extra), srcs))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-lpthread", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
