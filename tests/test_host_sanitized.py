"""The host side of the library under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): mesh validation, the threaded
geometry build, the CFL number, argument checks of every entry point and the
batch packing rules run in a library whose host code is instrumented, and
the ABI and batch-host tests must pass there with no sanitizer report.

The sanitized library is built once per source change (about two minutes
on eight cores) into ``paper_1608_03836_amd/_build_san``; the tests run in a
child process with the ASan runtime preloaded and the binding pointed at
that build."""

import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build_module():
    spec = importlib.util.spec_from_file_location(
        "_wadg_build", os.path.join(ROOT, "paper_1608_03836_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


@pytest.mark.timeout(900)
def test_host_code_is_clean_under_asan_and_ubsan():
    b = _build_module()
    try:
        runtime = b.sanitizer_runtime()
    except Exception as e:  # noqa: BLE001
        pytest.skip(f"no sanitizer runtime: {e}")
    lib = b.build_host_sanitized()
    env = dict(os.environ)
    env.update(LD_PRELOAD=runtime, WADG_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi.py"),
           os.path.join(ROOT, "tests", "test_batch_host.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
    # the child really loaded the instrumented build
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_" in nm and "__ubsan_" in nm
