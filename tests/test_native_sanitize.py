"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`build()` also compiles libqw with the sanitizers on its host code (device
code as in the product build) and links `tests/native/sanitize_driver.cpp`
against it. The driver calls the C ABI: on the CPU every entry point's
argument checks and error paths; on a GPU a short run of plans, jumps,
steps, reductions, autotuning with a schedule cache and a server on three
streams with cancellations and timed waits. A sanitizer report fails the run.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_DIR = os.path.join(ROOT, "paper_1603_06442_amd", "_build", "san")
DRIVER = os.path.join(SAN_DIR, "sanitize_driver")
SUPP = os.path.join(ROOT, "tests", "native", "lsan.supp")


def _run(mode, timeout, cwd):
    if not os.path.exists(DRIVER):
        pytest.skip("sanitizer build not present (run __graft_entry__.build())")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:detect_leaks=1:abort_on_error=0:exitcode=23"
    env["LSAN_OPTIONS"] = "suppressions=%s:print_suppressions=0" % SUPP
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    print("running", DRIVER, mode, flush=True)
    p = subprocess.run([DRIVER, mode], env=env, cwd=cwd, capture_output=True, text=True,
                       timeout=timeout)
    out = p.stdout + p.stderr
    print(out[-4000:])
    assert p.returncode == 0, out[-8000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out
    assert "ERROR: LeakSanitizer" not in out
    assert out.rstrip().endswith("OK") or "\nOK\n" in out


def test_host_paths_under_sanitizers(tmp_path):
    """No device needed: argument validation of every entry point and the
    error paths of plan and server creation."""
    _run("host", 120, str(tmp_path))


@pytest.mark.gpu
def test_device_run_under_host_sanitizers(tmp_path):
    # the driver writes its schedule cache file into its working directory
    _run("device", 300, str(tmp_path))
