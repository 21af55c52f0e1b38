"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its C
source and a driver that calls every entry point (tests/sanitize/) are built
with gcc -fsanitize=address,undefined and run; any finding aborts the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    build = subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fno-omit-frame-pointer",
                            "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-fast-math",
                            "-ffp-contract=off", "-o", exe, os.path.join(HERE, "sanitize", "oracle_driver.c"),
                            "-lm", "-lpthread"], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "oracle driver ok" in run.stdout
