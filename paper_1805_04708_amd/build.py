"""Build ``libjq.so`` (HIP, gfx950) in-tree with hipcc.

Every source under ``csrc/`` is compiled to an object file in ``_build/`` and
linked into ``paper_1805_04708_amd/libjq.so``.  ``build()`` always compiles
(it is the does-it-build check); ``ensure_built()`` compiles only when the
library is missing.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libjq.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
# no packed-FP32 instructions anywhere in device code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# the two-byte code must round every operation on its own to reproduce codes;
# the fused pass dispatches on wave-uniform op codes, so its branches need no
# structurisation (which would otherwise merge the whole register tile
# through chains of copy blocks)
_UNIFORM = ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]
# roctx ranges (JQ_ROCTX=1) come from the ROCm profiler SDK's marker library
LIBS = ["-lpthread", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
PER_FILE = {"kernels_compact.hip": ["-ffp-contract=off"] + _UNIFORM,
            "kernels_sv.hip": _UNIFORM, "batch.hip": _UNIFORM}


def _sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON + PER_FILE.get(src, [])
    if src.endswith(".hip"):
        cmd += DEVICE + ["-x", "hip"]
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(line for line in r.stderr.splitlines()
                     if "packed-fp32-ops" not in line and line.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{errs}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + LIBS
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


# Host sanitizer build: the same library with AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only (device code is built as
# usual), for the CPU tests; load it with the sanitizer runtime preloaded
# (see tests/test_sanitizers_cpu.py).
SAN_DIR = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libjq.so")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _compile_sanitized(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(SAN_DIR, src + ".o")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC"] + PER_FILE.get(src, []) + SAN_HOST
    if src.endswith(".hip"):
        cmd += DEVICE + ["-x", "hip"]
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-4000:]}")
    return obj


def build_sanitized() -> str:
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = _sources()
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile_sanitized, srcs))
    tmp = SAN_LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + SAN_HOST + ["-Xarch_host", "-shared-libsan",
                                                                              "-o", tmp] + objs + LIBS
    subprocess.check_call(cmd)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def sanitizer_runtime() -> str:
    """The AddressSanitizer runtime of the ROCm clang that built SAN_LIB."""
    r = subprocess.run([HIPCC, "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = hits[0] if hits else ""
    return path


def ensure_built() -> str:
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
