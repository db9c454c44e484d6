"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
a small driver (tests/native/oracle_sanitize_main.c) runs every entry point
of oracle/oracle.c (searches by brute force and cell list with one and
three threads, periodic and walled boxes, q, D, D^T, M, its diagonal,
Algorithm 1 for the three step rules, the adjoint's geometric terms), built
with gcc -fsanitize=address,undefined and no recovery; any invalid access,
leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(HERE, "native", "oracle_sanitize_main.c"), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "box 0:" in r.stdout and "box 1:" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
