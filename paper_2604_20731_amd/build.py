"""Build libcrv.so (HIP kernels for gfx950 + host runtime) in-tree with hipcc.

    python -m paper_2604_20731_amd.build              # libcrv.so
    python -m paper_2604_20731_amd.build --sanitize   # host sanitizer check

Every source is compiled to an object under csrc/_build (in parallel), then
linked into paper_2604_20731_amd/libcrv.so.  All device code is built with
the packed-FP32 instructions disabled.

--sanitize compiles the host side of every source with AddressSanitizer and
UndefinedBehaviorSanitizer (device code as usual, uninstrumented), links it
with the
csrc/abi_check.cpp driver into csrc/_build/asan/abi_check and runs it: the
C ABI's argument and configuration checks, which need no GPU.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libcrv.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = [
    "tables.cpp",
    "runtime.cpp",
    "k_fields.hip",
    "k_solve.hip",
    "k_mlp.hip",
    "k_mlp_mfma.hip",
    "k_galerkin.hip",
    "noalloc.hip",
]

ARCH = os.environ.get("CRV_OFFLOAD_ARCH", "gfx950")
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in ordinary VGPRs: no copies between the
    # accumulation registers and the VALU that applies tanh to every product
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wno-unused-result",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    hipcc = _hipcc()
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip") or src == "runtime.cpp":
        cmd = [hipcc, "-x", "hip", *HIP_FLAGS, "-I", INCLUDE, "-c", path, "-o", obj]
    else:  # plain C++ host tables: no FMA contraction, so float64 tables are reproducible
        cmd = [shutil.which("g++") or "g++", "-O2", "-fPIC", "-std=c++17", "-ffp-contract=off",
               "-I", INCLUDE, "-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _clangxx() -> str:
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("clang++ not found")


def build_sanitized(jobs: int | None = None) -> int:
    """Host-only sanitized build of the library plus the ABI driver; runs the
    driver and returns its exit status (0: every check passed, no report)."""
    out = os.path.join(BUILD, "asan")
    os.makedirs(out, exist_ok=True)
    hipcc = _hipcc()

    def one(src):
        obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
        path = os.path.join(CSRC, src)
        if src.endswith(".hip") or src == "runtime.cpp":
            cmd = [hipcc, "-x", "hip", *HIP_FLAGS, "-Xarch_host", "-g", *SAN_FLAGS, "-I", INCLUDE,
                   "-c", path, "-o", obj]
        else:
            cmd = [hipcc, "-x", "c++", "-O1", "-g", "-fPIC", "-std=c++17", *SAN_FLAGS, "-I",
                   INCLUDE, "-c", path, "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stderr}")
        return obj

    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, SOURCES + ["abi_check.cpp"]))
    exe = os.path.join(out, "abi_check")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    link = [_clangxx(), "-fsanitize=address,undefined", "-o", exe, *objs,
            f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{rocm}/lib"]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(link)}\n{res.stderr}")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env)
    sys.stdout.write(run.stdout)
    sys.stderr.write(run.stderr)
    return run.returncode


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        sys.exit(build_sanitized())
    build(verbose=True)
    sys.exit(0)
