"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Builds the library with the sanitizers on its host code (planner, gate
lowering, tuning table and cache file, runtime validation) and the oracle's
C code with them too, then runs the host-side test files against those
builds in a child process with the sanitizer runtime preloaded: any memory
error or undefined behaviour aborts the child and fails this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_plan_cpu.py", "tests/test_abi_cpu.py", "tests/test_tuning_cpu.py",
              "tests/test_oracle_pins.py", "tests/test_oracle_paper_cpu.py", "tests/test_oracle_measure.py",
              "tests/test_oracle_noise.py", "tests/test_oracle_shor.py", "tests/test_oracle_aux.py"]


def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    from oracle import build as OB
    from paper_1805_04708_amd import build as B

    jq_lib = B.build_sanitized()
    oracle_lib, pc_lib = OB.build_sanitized()
    rt = B.sanitizer_runtime()
    if not rt:
        pytest.skip("no AddressSanitizer runtime in this ROCm installation")
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "JQ_LIB": jq_lib, "JQ_ORACLE_LIB": oracle_lib, "JQ_PAPERCPU_LIB": pc_lib,
        "JQ_TUNE_CACHE": str(tmp_path / "tuning.json"),
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
                       + HOST_TESTS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout[-3000:] + "\n" + r.stderr[-6000:])
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
