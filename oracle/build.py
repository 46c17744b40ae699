"""Compile the oracle's C code into ``oracle/liboracle.so`` with gcc.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Building the checker
is not using it: the package's ``build()`` calls this so the tests find it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jq_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the paper's OpenMP method (Sec. 3.1), the multi-core CPU baseline
PC_SRC = os.path.join(HERE, "paper_cpu.c")
PC_LIB = os.path.join(HERE, "libpapercpu.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-Wall", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    if force or not os.path.exists(PC_LIB) or os.path.getmtime(PC_LIB) < os.path.getmtime(PC_SRC):
        tmp = PC_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-Wall", "-shared", "-fPIC", "-o", tmp, PC_SRC])
        os.replace(tmp, PC_LIB)
    return LIB


# Host sanitizer build of both libraries (AddressSanitizer and
# UndefinedBehaviorSanitizer, ROCm's clang so that one sanitizer runtime
# serves them and the GPU library's sanitizer build in one process).
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_DIR = os.path.join(os.path.dirname(HERE), "_build", "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "liboracle.so")
SAN_PC_LIB = os.path.join(SAN_DIR, "libpapercpu.so")
_SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
        "-ffp-contract=off", "-std=c99", "-D_DEFAULT_SOURCE", "-shared", "-fPIC"]


def build_sanitized() -> tuple:
    os.makedirs(SAN_DIR, exist_ok=True)
    subprocess.check_call([CLANG] + _SAN + ["-o", SAN_LIB, SRC, "-lm"])
    subprocess.check_call([CLANG] + _SAN + ["-fopenmp", "-o", SAN_PC_LIB, PC_SRC, "-L/opt/rocm/llvm/lib",
                                            "-Wl,-rpath,/opt/rocm/llvm/lib"])
    return SAN_LIB, SAN_PC_LIB


if __name__ == "__main__":
    print(build())
