"""Build tests/host_sanitize/_build/driver: the C-ABI driver (driver.cpp)
linked with the library's host code instrumented by AddressSanitizer and
UndefinedBehaviorSanitizer.  Device code is not instrumented: atns.cpp is
compiled with the sanitizer flags for its host pass only, and the kernel
objects of the regular build (paper_2506_03027_amd/_build) are linked as
they are.  Run `python tests/host_sanitize/build.py` after the library build."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2506_03027_amd", "csrc")
LIBBUILD = os.path.join(ROOT, "paper_2506_03027_amd", "_build")
OUT = os.path.join(HERE, "_build")
DRIVER = os.path.join(OUT, "driver")
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
SAN = ["address", "undefined"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))


def build():
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    # the library's host code, sanitized on the host pass only
    host_san = []
    for s in SAN:
        host_san += ["-Xarch_host", "-fsanitize=" + s]
    host_san += ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
    _run([os.path.join(ROCM, "bin", "hipcc"), "-O2", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
         + host_san + inc + ["-x", "hip", "-c", os.path.join(CSRC, "atns.cpp"),
                             "-o", os.path.join(OUT, "atns_san.o")])
    # plain C++ parts: host tables and the driver
    cxx = [CLANG, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include")] + ["-fsanitize=" + ",".join(SAN)] + inc
    _run(cxx + ["-c", os.path.join(CSRC, "coeffs.cpp"), "-o", os.path.join(OUT, "coeffs_san.o")])
    _run(cxx + ["-c", os.path.join(HERE, "driver.cpp"), "-o", os.path.join(OUT, "driver.o")])
    kernels = [os.path.join(LIBBUILD, f) for f in sorted(os.listdir(LIBBUILD))
               if f.endswith(".o") and f not in ("atns.o", "coeffs.o")]
    _run([CLANG, "-fsanitize=" + ",".join(SAN), "-o", DRIVER, os.path.join(OUT, "driver.o"),
          os.path.join(OUT, "atns_san.o"), os.path.join(OUT, "coeffs_san.o")] + kernels
         + ["-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    return DRIVER


if __name__ == "__main__":
    print("built", build())
    sys.exit(0)
