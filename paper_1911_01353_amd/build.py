"""Builds the HIP library ``libjerk.so`` in-tree for gfx950.

Usage: ``python -m paper_1911_01353_amd.build`` (or ``build()`` from Python).
Every source is recompiled on each call; objects go to ``_build/`` next to
this file and the library to ``libjerk.so`` beside it.

``--sanitize`` builds ``libjerk_asan.so`` instead, its host code instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (device code is not), and
``--sanitize --run-tests`` then runs the CPU test suite against it (the ASan
runtime preloaded into Python, ``JERK_LIBRARY`` pointing the binding at it):
plan arithmetic, argument validation of every entry point and the serving
scheduler's dry-run mode, all on the host.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libjerk.so")
ASAN_OUT_DIR = os.path.join(HERE, "_build_asan")
ASAN_LIB = os.path.join(HERE, "libjerk_asan.so")
# host-side only: -Xarch_host keeps the sanitizers out of the device code
SANITIZE = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
ARCH = "gfx950"

# Packed FP32 instructions are disabled for all device code.
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include")]


def _hipcc() -> str:
    cand = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cand):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libjerk.so")
    return cand


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(ASAN_OUT_DIR if sanitize else OUT_DIR, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *COMMON, *(SANITIZE if sanitize else []), "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(line for line in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in line)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    if out.strip():
        print(out, file=sys.stderr)
    return obj


def build(verbose: bool = True, sanitize: bool = False) -> str:
    out_dir, lib = (ASAN_OUT_DIR, ASAN_LIB) if sanitize else (OUT_DIR, LIB)
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), srcs))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if sanitize:
        cmd[1:1] = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}{res.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}", file=sys.stderr)
    if sanitize:
        return lib
    demo = build_c_demo()
    if verbose:
        print(f"built {demo}", file=sys.stderr)
    probe = build_peakprobe()
    if verbose:
        print(f"built {probe}", file=sys.stderr)
    return LIB


PEAKPROBE_SRC = os.path.join(HERE, "peakprobe.hip")
PEAKPROBE = os.path.join(HERE, "peakprobe")


def build_peakprobe() -> str:
    """The arithmetic-ceiling probe bench.py runs (MFMA bf16 and FP32 FMA loops)."""
    cmd = [_hipcc(), *COMMON, PEAKPROBE_SRC, "-o", PEAKPROBE + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"peak probe build failed: {' '.join(cmd)}\n{res.stdout}{res.stderr}")
    os.replace(PEAKPROBE + ".tmp", PEAKPROBE)
    return PEAKPROBE


C_DEMO_SRC = os.path.join(HERE, "..", "tests", "c_abi", "jerk_demo.c")
C_DEMO = os.path.join(HERE, "..", "tests", "c_abi", "jerk_demo")


def build_c_demo() -> str:
    """The C caller used by the tests (plain C against include/jerk.h and libjerk.so)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(_hipcc())))
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("a C compiler (gcc) is required to build the C demo")
    cmd = [cc, "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(HERE, "..", "include"), "-I", os.path.join(rocm, "include"),
           C_DEMO_SRC, "-o", C_DEMO + ".tmp", "-L", HERE, "-ljerk", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1911_01353_amd", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"C demo build failed: {' '.join(cmd)}\n{res.stdout}{res.stderr}")
    os.replace(C_DEMO + ".tmp", C_DEMO)
    return os.path.normpath(C_DEMO)


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime that hipcc links against (preloaded into Python)."""
    res = subprocess.run([_hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        rocm = os.path.dirname(os.path.dirname(os.path.realpath(_hipcc())))
        import glob
        found = glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so"))
        if not found:
            raise RuntimeError("AddressSanitizer runtime not found")
        path = found[0]
    return path


def run_sanitized_tests(pytest_args=()) -> int:
    """Runs the CPU test suite with the sanitized library (ASan + UBSan on the host code)."""
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan_runtime()
    env["JERK_LIBRARY"] = ASAN_LIB
    # Python and the HIP runtime are not instrumented: no leak report, stop at the first error
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", os.path.join(HERE, "..", "tests"), "-q", "-m", "not gpu", *pytest_args]
    return subprocess.run(cmd, env=env).returncode


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sanitize", action="store_true", help="build libjerk_asan.so (host ASan + UBSan)")
    ap.add_argument("--run-tests", action="store_true", help="with --sanitize: run the CPU tests against it")
    a = ap.parse_args()
    if a.sanitize:
        build(sanitize=True)
        if a.run_tests:
            sys.exit(run_sanitized_tests())
    else:
        build()
