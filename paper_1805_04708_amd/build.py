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
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
