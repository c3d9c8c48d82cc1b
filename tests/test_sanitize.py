"""The CPU oracle and the input generators under AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only): tests/sanitize/driver.c
runs every oracle entry point on small seeded graphs; any invalid access or
undefined operation makes the run fail."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_and_generators_under_sanitizers(tmp_path):
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "sanitize", "driver.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "synth", "synth.c"),
           "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="3")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, f"sanitized run failed:\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    assert "sanitized run ok" in r.stdout
