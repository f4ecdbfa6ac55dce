"""Build libspx.so (the HIP library behind include/spx.h) for gfx950.

Every source under csrc/ is compiled by hipcc to an object in _build/ (in
parallel), then linked into paper_2006_14290_amd/libspx.so. Always rebuilds.

build_hostsan() builds a second copy, libspx_hostsan.so, whose host code is
instrumented with AddressSanitizer and UBSan (device code is compiled as
usual), and the test driver tests/sanitize/abi_driver_hostsan linked against
it, which the sanitizer tests run.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libspx.so")
LIB_HOSTSAN = os.path.join(HERE, "libspx_hostsan.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
DRIVER_SRC = os.path.join(os.path.dirname(HERE), "tests", "sanitize", "abi_driver.cpp")
DRIVER_HOSTSAN = os.path.join(os.path.dirname(HERE), "tests", "sanitize", "abi_driver_hostsan")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-x", "hip",
    # packed-FP32 instructions are kept out of the device code on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I" + INCLUDE,
]

# host-side instrumentation only: every sanitizer option is routed to the
# host compilation, so the gfx950 code objects are the ordinary ones
HOSTSAN_FLAGS = [
    "-g", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str, outdir: str = BUILD, extra=()) -> str:
    obj = os.path.join(outdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    errs = [l for l in r.stderr.splitlines() if "warning" in l and "packed-fp32-ops" not in l]
    if errs:
        sys.stderr.write("\n".join(errs) + "\n")
    return obj


def _link(objs, out: str):
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, sources()))
    _link(objs, LIB)
    return LIB


def build_hostsan(jobs: int = 8) -> str:
    """libspx_hostsan.so and the ABI test driver, both with ASan + UBSan on
    the host side. The sanitizer runtime is linked into the driver; the
    library resolves its instrumentation hooks against it at load time."""
    out = os.path.join(BUILD, "hostsan")
    os.makedirs(out, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, out, HOSTSAN_FLAGS), sources()))
    _link(objs, LIB_HOSTSAN)
    tmp = DRIVER_HOSTSAN + ".tmp"
    cmd = [CLANGXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I" + INCLUDE,
           "-I" + os.path.join(ROCM, "include"), DRIVER_SRC, "-o", tmp, LIB_HOSTSAN,
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lpthread",
           "-Wl,-rpath," + HERE, "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver build failed:\n{r.stderr}")
    os.replace(tmp, DRIVER_HOSTSAN)
    return LIB_HOSTSAN


if __name__ == "__main__":
    print(build())
    if len(sys.argv) > 1 and sys.argv[1] == "hostsan":
        print(build_hostsan())
