"""Build libfdot.so (HIP for gfx950) in-tree, and the input generator's
device library.  Used by __graft_entry__.build(); run as a script to rebuild.

--sanitize builds host-instrumented copies of the library and of the oracle
(AddressSanitizer and UndefinedBehaviorSanitizer on the host code; device
code is compiled as usual) under _build/san/, then runs the CPU test suite
against them in a child process with the sanitizer runtime preloaded; any
report fails the run."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfdot.so")
SYNTH_SRC = os.path.join(ROOT, "synth", "synth.hip")
SYNTH_LIB = os.path.join(ROOT, "synth", "libsynth.so")

ARCH = os.environ.get("FDOT_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for every HIP translation unit.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function", "-Wno-unused-result"]

SOURCES = ["host_field.cpp", "runtime.cpp", "dot_kernels.hip", "gemm_kernels.hip",
           "gemm_mfma.hip", "elementwise.hip", "ext_field.hip", "many_mixed.hip", "server.cpp",
           "calibrate.hip", "noalloc.hip", "validate.hip"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON
    if src.endswith(".hip"):
        cmd += ["-x", "hip"] + DEVICE_FLAGS
    else:
        cmd += ["-D__HIP_PLATFORM_AMD__"]
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    # input generator (separate library: not part of the product)
    tmp = SYNTH_LIB + ".tmp"
    cmd = [HIPCC, "-O3", "-fPIC", "-shared", f"--offload-arch={ARCH}", "-x", "hip"] + DEVICE_FLAGS + \
          [SYNTH_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"synth build failed:\n{r.stderr}")
    os.replace(tmp, SYNTH_LIB)
    if verbose:
        print("built", LIB, "and", SYNTH_LIB)
    return LIB


SAN_DIR = os.path.join(BUILD, "san")
LLVM_BIN = "/opt/rocm/lib/llvm/bin"
# host-side instrumentation only: each -fsanitize= applies to the host pass
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def asan_runtime() -> str:
    r = subprocess.run([os.path.join(LLVM_BIN, "clang"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.exists(path):
        raise RuntimeError("the clang AddressSanitizer runtime was not found")
    return path


def _compile_san(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(SAN_DIR, src + ".o")
    cmd = [HIPCC] + COMMON + ["-g", "-O1"] + SAN_HOST
    if src.endswith(".hip"):
        cmd += ["-x", "hip"] + DEVICE_FLAGS
    else:
        cmd += ["-D__HIP_PLATFORM_AMD__"]
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build_sanitized(verbose: bool = False):
    """Host-instrumented libfdot.so and liboracle.so under _build/san/."""
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile_san, srcs))
    lib = os.path.join(SAN_DIR, "libfdot.so")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan", "-o", lib] + objs + \
          ["-lpthread", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    orc = os.path.join(SAN_DIR, "liboracle.so")
    cmd = [os.path.join(LLVM_BIN, "clang"), "-g", "-O1", "-std=c11", "-fPIC", "-shared",
           "-shared-libsan", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-fopenmp", "-Wl,-rpath," + os.path.join(LLVM_BIN, "..", "lib"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-o", orc, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle build failed: {' '.join(cmd)}\n{r.stderr}")
    if verbose:
        print("built", lib, "and", orc)
    return lib, orc


def run_sanitized(pytest_args=()) -> int:
    """The CPU test suite against the instrumented libraries (child process,
    sanitizer runtime preloaded, leak checks off: the interpreter's own
    allocations are not ours)."""
    lib, orc = build_sanitized(verbose=True)
    env = dict(os.environ)
    env.update({"FDOT_LIB": lib, "ORACLE_LIB": orc, "LD_PRELOAD": asan_runtime(),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    cmd = [sys.executable, "-m", "pytest", "tests", "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
    return subprocess.call(cmd + list(pytest_args), cwd=ROOT, env=env)


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        sys.exit(run_sanitized([a for a in sys.argv[1:] if a != "--sanitize"]))
    build(verbose=True)
    sys.exit(0)
