"""Build tests/bin/host_sanitize_check: the host-side sanitizer driver
(tests/host_sanitize_check.c) linked with libcorr's host sources (corr.cpp,
sched.cpp) compiled under AddressSanitizer and UndefinedBehaviorSanitizer.

Only the host side is instrumented: on each hipcc line every -fsanitize
option follows -Xarch_host, and the device code of the other translation
units is the regular build's (_build/*.o).  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_0906_1887_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(ROOT, "_build")
BIN_DIR = os.path.join(HERE, "bin")
EXE = os.path.join(BIN_DIR, "host_sanitize_check")
ROCM = "/opt/rocm"
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
SANITIZED = ("corr.cpp", "sched.cpp")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{cmd[0]} failed:\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}")


def build() -> str:
    """Compile the sanitized host objects and link the driver; returns its path."""
    if not all(os.path.exists(os.path.join(OBJ, "corr_" + os.path.splitext(s)[0] + ".o"))
               for s in ("xengine_mfma.hip", "accum.hip")):
        from paper_0906_1887_amd import build as corr_build
        corr_build.build()
    os.makedirs(BIN_DIR, exist_ok=True)
    tmp = os.path.join(BIN_DIR, "obj")
    os.makedirs(tmp, exist_ok=True)
    objs = []
    for src in SANITIZED:
        o = os.path.join(tmp, os.path.splitext(src)[0] + "_san.o")
        _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", INCLUDE, "-I", CSRC, *HOST_SAN, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    drv = os.path.join(tmp, "host_sanitize_check.o")
    _run([CLANG, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
          "-I", INCLUDE, "-c", os.path.join(HERE, "host_sanitize_check.c"), "-o", drv])
    skip = {"corr_" + os.path.splitext(s)[0] + ".o" for s in SANITIZED}
    rest = sorted(os.path.join(OBJ, f) for f in os.listdir(OBJ) if f.endswith(".o") and f not in skip)
    _run([CLANGXX, "-fsanitize=address,undefined", "-o", EXE + ".tmp", drv, *objs, *rest,
          "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build())
