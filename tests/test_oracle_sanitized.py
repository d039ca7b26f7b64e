"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is built a second time with gcc's address and undefined-behaviour
sanitizers (host code only; the oracle has no GPU code) and the pins run
against that build in a child process, with the sanitizer runtime preloaded
into the interpreter.  Any out-of-bounds access, use after free or undefined
operation in the oracle aborts the child, so the pins fail.  CPU only.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dem_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")
SLOW = "tests/test_oracle_pins.py::test_energy_drift_plain_fp64_workload"


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "libdem_oracle_sanitized.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fPIC", "-shared", SRC, "-o", lib,
                    "-lm"], check=True, capture_output=True)
    env = dict(os.environ, DEM_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", PINS, "-q", "-x", "-p", "no:cacheprovider", "--deselect", SLOW],
                       env=env, capture_output=True, text=True, cwd=ROOT, timeout=900)
    tail = "\n".join((r.stdout + r.stderr).strip().splitlines()[-20:])
    assert r.returncode == 0, f"pins under the sanitizers failed:\n{tail}"
    assert " passed" in r.stdout and "error" not in r.stdout.lower().split(" passed")[-1]
