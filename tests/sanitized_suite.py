"""Run the CPU test suite (-m "not gpu") against host builds instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer: the library's host code (plan,
C ABI, launchers; device code unchanged) and the oracle's C sums.

    python tests/sanitized_suite.py [extra pytest arguments]

Builds into paper_2506_23568_amd/csrc/_build/sanitized/ and oracle/_build/, then
runs pytest with the clang ASan runtime preloaded.  CPU only: no test that runs
here touches a GPU.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_23568_amd", "csrc")
OUT = os.path.join(CSRC, "_build", "sanitized")
ORACLE_OUT = os.path.join(ROOT, "oracle", "_build")
LLVM = "/opt/rocm/llvm/bin"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["address", "undefined"]


def host_san_flags():
    """-Xarch_host before each sanitizer flag: host code only."""
    out = []
    for s in SAN:
        out += ["-Xarch_host", "-fsanitize=" + s]
    return out + ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build():
    os.makedirs(OUT, exist_ok=True)
    os.makedirs(ORACLE_OUT, exist_ok=True)
    base = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include")]
    objs = []
    for src in ("api.cpp", "plan.cpp", "kernels.hip", "kernels_adjoint.hip", "kernels_metrics.hip"):
        obj = os.path.join(OUT, src + ".o")
        subprocess.check_call([HIPCC] + base + host_san_flags() +
                              ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    lib = os.path.join(OUT, "libhhffbp.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib] + objs +
                          host_san_flags() + ["-lpthread"])
    olib = os.path.join(ORACLE_OUT, "liboracle_sanitized.so")
    subprocess.check_call([os.path.join(LLVM, "clang"), "-O1", "-g", "-fno-fast-math",
                           "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-fsanitize=" + ",".join(SAN), "-fno-omit-frame-pointer",
                           "-fno-sanitize-recover=all",
                           os.path.join(ROOT, "oracle", "oracle.c"), "-o", olib, "-lm"])
    return lib, olib


def main():
    lib, olib = build()
    rt = subprocess.check_output([os.path.join(LLVM, "clang"),
                                  "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    env = dict(os.environ, HHFFBP_LIBRARY=lib, ORACLE_LIBRARY=olib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               LD_LIBRARY_PATH="/opt/rocm/llvm/lib:" + os.environ.get("LD_LIBRARY_PATH", ""))
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-x", "-q",
           "-p", "no:xdist"] + sys.argv[1:]
    print(" ".join(cmd), flush=True)
    return subprocess.call(cmd, env=env, cwd=ROOT)


if __name__ == "__main__":
    sys.exit(main())
