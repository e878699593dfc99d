"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
driver (tests/sanitize/oracle_driver.c) runs every oracle entry point (random
numbers, the three parameterisations, probabilities for Pauli settings and
POVMs, both likelihoods, the network forward pass, chains with and without
delayed acceptance, traces, records, pooling) and must finish with no report
(any report aborts the process with a non-zero status)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    src = os.path.join(HERE, "sanitize", "oracle_driver.c")
    flags = ["-O1", "-g", "-std=gnu11", "-fopenmp", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(["gcc", *flags, "-o", str(exe), src, "-lm"], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle driver done" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
