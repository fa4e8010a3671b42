"""Build libnssdoa.so for gfx950 with hipcc (used by ``__graft_entry__.build``).

Every HIP source under csrc/ is compiled to an object in ``_build/`` at the repository root and
linked into ``paper_2007_14135_amd/libnssdoa.so``.  Packed FP32 instructions are disabled for
device code (``-packed-fp32-ops``); hipcc's host pass warns that it does not know the feature,
which is harmless.
"""

from __future__ import annotations

import concurrent.futures
import glob
import os
import shlex
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libnssdoa.so")
ARCH = os.environ.get("NSSDOA_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


# Per-source flags.  The scans keep their matrix-core accumulators in ordinary VGPRs (the
# epilogue reads them with plain vector instructions instead of accvgpr copies).
SOURCE_FLAGS = {"scan_f32.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}

# Host AddressSanitizer copy of the library and its C ABI driver (tests/asan): host code
# instrumented, device code as in the product build.
ASAN_DIR = os.path.join(ROOT, "tests", "asan", "_build")
ASAN_LIB = os.path.join(ASAN_DIR, "libnssdoa_asan.so")
ASAN_DRIVER = os.path.join(ASAN_DIR, "abi_driver")
ASAN_HOST_FLAGS = shlex.split("-Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer -Xarch_host -g")
CLANGXX = os.environ.get("NSSDOA_CLANGXX", "/opt/rocm/llvm/bin/clang++")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(src: str, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + CFLAGS + SOURCE_FLAGS.get(os.path.basename(src), []) + list(extra) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every csrc/*.hip and link libnssdoa.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s failed:\n%s\n%s" % (what, " ".join(cmd), r.stderr))


def build_asan(verbose: bool = False) -> str:
    """Host-ASan libnssdoa_asan.so and the driver tests/asan/abi_driver.cpp linked against it
    (with the ASan runtime in the executable); returns the driver's path."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, ASAN_DIR, ASAN_HOST_FLAGS), srcs))
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", ASAN_LIB] + objs, "ASan library link")
    drv = os.path.join(ROOT, "tests", "asan", "abi_driver.cpp")
    dobj = os.path.join(ASAN_DIR, "abi_driver.o")
    san = shlex.split("-fsanitize=address -fno-omit-frame-pointer -g")
    _run([CLANGXX, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
          "-I", INCLUDE] + san + ["-c", drv, "-o", dobj], "ASan driver compile")
    _run([CLANGXX] + san + [dobj, "-o", ASAN_DRIVER, "-L", ASAN_DIR, "-lnssdoa_asan",
                            "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                            "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(ROCM, "lib")],
         "ASan driver link")
    if verbose:
        print("built", ASAN_DRIVER)
    return ASAN_DRIVER


if __name__ == "__main__":
    build(verbose=True)
    if len(sys.argv) > 1 and sys.argv[1] == "asan":
        build_asan(verbose=True)
    sys.exit(0)
