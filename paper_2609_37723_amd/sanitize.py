"""Host-side sanitizer runs of the CPU test suites (no GPU needed).

1. AddressSanitizer + UndefinedBehaviorSanitizer on the library's host code (argument
   checks, planning, the serving scheduler with its fake executor): build.py's
   ``sanitize="address"`` build, loaded through NUC_LIBRARY with the clang ASan runtime
   preloaded, under tests/test_abi_cpu.py and tests/test_server_cpu.py.
2. ThreadSanitizer on the same host code (the server's scheduler thread against the
   submitting and waiting threads): ``sanitize="thread"``, with the clang TSan runtime
   preloaded, under tests/test_server_cpu.py.
3. AddressSanitizer + UndefinedBehaviorSanitizer on the FP64 oracle (gcc), loaded through
   ORACLE_LIBRARY with gcc's libasan preloaded, under the oracle's pin tests.

Usage: ``python paper_2609_37723_amd/sanitize.py [address] [thread] [oracle]`` (all three by
default). Exits non-zero if any run fails or a sanitizer reports.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def clang_runtime(name: str) -> str:
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.%s-x86_64.so" % name))
    if not hits:
        raise FileNotFoundError("clang %s runtime not found under /opt/rocm/llvm" % name)
    return hits[-1]


def gcc_runtime(name: str) -> str:
    return subprocess.check_output(["gcc", "-print-file-name=lib%s.so" % name], text=True).strip()


def run(label: str, env: dict, tests: list) -> bool:
    e = dict(os.environ)
    e.update(env)
    # -s: a sanitizer report goes straight to stderr (pytest's capture would hold it back if the
    # process ends on it)
    cmd = [sys.executable, "-m", "pytest", "-q", "-s", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + tests
    print("[sanitize] %s: %s" % (label, " ".join("%s=%s" % kv for kv in env.items())), flush=True)
    r = subprocess.run(cmd, cwd=ROOT, env=e, capture_output=True, text=True)
    out = r.stdout + r.stderr
    reported = any(s in out for s in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer",
                                      "ERROR: ThreadSanitizer", "ERROR: LeakSanitizer"))
    tail = [l for l in out.strip().splitlines() if l.strip()][-3:]
    print("[sanitize] %s: exit %d, sanitizer report: %s; %s" % (label, r.returncode, "yes" if reported else "none",
                                                             " | ".join(tail)), flush=True)
    if reported:
        print(out, flush=True)
    return r.returncode == 0 and not reported


def main(which):
    from paper_2609_37723_amd import build
    ok = True
    if "address" in which:
        lib = build.build(sanitize="address")
        ok &= run("ASan+UBSan, library host code",
                  {"NUC_LIBRARY": lib, "LD_PRELOAD": clang_runtime("asan"),
                   "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
                   "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"},
                  ["tests/test_abi_cpu.py", "tests/test_server_cpu.py"])
    if "thread" in which:
        lib = build.build(sanitize="thread")
        ok &= run("TSan, library host code (server threads)",
                  {"NUC_LIBRARY": lib, "LD_PRELOAD": clang_runtime("tsan"),
                   "TSAN_OPTIONS": "halt_on_error=1:report_signal_unsafe=0"},
                  ["tests/test_server_cpu.py"])
    if "oracle" in which:
        import oracle
        lib = oracle.build(sanitize=True)
        ok &= run("ASan+UBSan, oracle",
                  {"ORACLE_LIBRARY": lib, "LD_PRELOAD": gcc_runtime("asan"),
                   "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1",
                   "OMP_NUM_THREADS": "4"},
                  ["tests/test_oracle_elementals.py", "tests/test_oracle_correlator.py",
                   "tests/test_oracle_spin.py"])
    print("[sanitize] %s" % ("all clean" if ok else "FAILED"), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:] or ["address", "thread", "oracle"]))
