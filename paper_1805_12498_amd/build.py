"""Build libhafgpu.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1805_12498_amd.build

Each source is compiled to an object in ``_build/`` (in parallel), then linked
into ``paper_1805_12498_amd/libhafgpu.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhafgpu.so")

ARCH = os.environ.get("HAFGPU_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SOURCES = [
    "haf_kernels_lds.hip",
    "haf_kernels_reg.hip",
    "haf_kernels_series.hip",
    "haf_noalloc.hip",
    "haf_kernels_modp.hip",
    "haf_kernels_dd.hip",
    "haf_kernels_lowrank.hip",
    "haf_runtime.cpp",
    "haf_batched.cpp",
    "haf_server.cpp",
    "haf_exact.cpp",
]
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # code object v5: loadable by the HIP runtime that PyTorch bundles as well as by /opt/rocm's
    "-mcode-object-version=5",
    # packed FP32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# sources whose arithmetic must not be contracted into fused multiply-adds
# (double-double error-free transformations)
NO_CONTRACT = {"haf_kernels_dd.hip"}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    extra = ["-ffp-contract=off"] if src in NO_CONTRACT else []
    cmd = [hipcc()] + HIP_FLAGS + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    workers = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    # roctx: named host ranges for rocprofv3 --marker-trace (no-ops without a tool)
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        "-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_host_sanitized(out_dir: str) -> str:
    """The library with its host code under AddressSanitizer and
    UndefinedBehaviorSanitizer (device code unsanitized and unoptimised, to build
    fast), into out_dir/libhafgpu_host_asan.so: for CPU tests of the host-side logic
    (planner, configuration, argument checks, error paths).  A process that loads
    it must preload the sanitizer runtime (asan_runtime())."""
    os.makedirs(out_dir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_device", "-O0",
             "-I" + INCLUDE, "-I" + CSRC] + san

    def one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + flags + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
        return obj

    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(min(len(srcs), max(1, min(8, os.cpu_count() or 1)))) as ex:
        objs = list(ex.map(one, srcs))
    lib = os.path.join(out_dir, "libhafgpu_host_asan.so")
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-shared-libsan"] + san + [
        "-o", lib] + objs + ["-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx",
                             "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return lib


def asan_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to preload)."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        hits = sorted(glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "*", "libclang_rt.asan-x86_64.so")))
        path = hits[-1] if hits else ""
    return path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
