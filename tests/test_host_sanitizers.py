"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
FP64 oracle (oracle/lbm_oracle.c, with OpenMP) and the library's lattice
builder and pull-table checks (csrc/lattice.cpp) are each built with
-fsanitize=address,undefined into a driver of their own
(tests/sanitize/*_driver.*) and run on small random boxes in every boundary
mode. A sanitizer report, or a failed conservation / bijection / decoding
check in a driver, fails the test. Host compilers only (gcc, g++)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _build_and_run(cmd, exe):
    subprocess.run(cmd, check=True, capture_output=True, text=True, cwd=os.path.dirname(exe))
    env = dict(ENV)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 failures" in out and "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _build_and_run(["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off"] + SAN +
                   ["-o", exe, os.path.join(ROOT, "oracle", "lbm_oracle.c"),
                    os.path.join(HERE, "sanitize", "oracle_driver.c"), "-lm"], exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_lattice_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "lattice_san")
    _build_and_run(["g++", "-std=c++17", "-pthread"] + SAN +
                   ["-I", os.path.join(ROOT, "include"), "-o", exe,
                    os.path.join(ROOT, "paper_1806_10589_amd", "csrc", "lattice.cpp"),
                    os.path.join(HERE, "sanitize", "lattice_driver.cpp")], exe)
