"""Sanitizer build of the CPU code: the oracle (oracle/sakura_oracle.c) and the
host build of the device pair solver (tests/solver_host_shim.cpp) compiled
with AddressSanitizer and UndefinedBehaviorSanitizer (every report fatal) and
run by tests/sanitize_driver.cpp on small seeded inputs, ragged sizes, massless
particles, every solver variant, composition scheme and the hybrid, error
paths and random Kepler problems of every kind.  Host code only: nothing here
is built for or runs on the GPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


@pytest.mark.slow
def test_oracle_and_host_solver_under_asan_ubsan(tmp_path):
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "sanitized")
    subprocess.check_call(["gcc", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp",
                           *SAN, "-c", os.path.join(ROOT, "oracle", "sakura_oracle.c"),
                           "-o", obj])
    subprocess.check_call(["g++", "-std=c++17", "-fopenmp", *SAN,
                           os.path.join(HERE, "sanitize_driver.cpp"),
                           os.path.join(HERE, "solver_host_shim.cpp"), obj, "-o", exe, "-lm"])
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1:"
                            "verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "SANITIZED_RUN_OK" in p.stdout
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
