"""The library's host runtime under AddressSanitizer and
UndefinedBehaviorSanitizer on the GPU: tests/sanitize/host_driver.cpp calls
every C entry point (validation and its allocation-free variant, FK,
NEAREST, samples, plans with and without history, rewiring, replanning, a
batch, a server with four requests, error paths); the build step links it
with every library source, the sanitizers on the host code only.  Any
finding, or a leak outside the HIP/HSA runtimes, fails the run."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "sanitize", "host_driver_asan")


def test_host_runtime_under_asan_ubsan():
    assert os.path.exists(EXE), "sanitized driver missing: run the build step (__graft_entry__.build())"
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:halt_on_error=1",
               LSAN_OPTIONS="suppressions=" + os.path.join(HERE, "sanitize", "lsan.supp"),
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    print("[sanitize] host driver", flush=True)
    run = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=240)
    print(run.stdout[-2000:], run.stderr[-4000:], flush=True)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-6000:]
    assert "host driver ok" in run.stdout
