"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The library is rebuilt with both sanitizers on its host code only (device code
as usual) into a temporary directory, and the C-ABI tests, which drive the
host validation of every entry point (invalid problems, bad arguments, null
handles, duplicate detection, status strings), run against it in a child
process that preloads the shared sanitizer runtime.  Any sanitizer report
fails the run (halt_on_error).  Leak detection is off: the Python interpreter
itself holds memory until exit.
"""

import os
import shutil
import subprocess
import sys

import pytest

from paper_2501_13385_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

RUNNER = """
import sys
import paper_2501_13385_amd._lib as lib
lib.LIB_PATH = sys.argv[1]
import pytest
sys.exit(pytest.main(["-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", sys.argv[2]]))
"""


def test_host_validation_is_clean_under_asan_and_ubsan(tmp_path):
    try:
        B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    runtime = B.sanitizer_runtime()
    if not runtime or not os.path.exists(runtime):
        pytest.skip("no shared ASan runtime next to the compiler")
    lib = B.build_host_sanitized(str(tmp_path))
    # the host code is instrumented by both sanitizers
    nm = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True)
    if nm.returncode == 0:
        assert "__asan_report_load" in nm.stdout and "__ubsan_handle_" in nm.stdout
    env = dict(os.environ)
    # the sanitizer runtime first, anything already preloaded kept after it
    env["LD_PRELOAD"] = runtime + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    res = subprocess.run([sys.executable, "-c", RUNNER, lib, os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    # the child really ran the sanitized build
    assert "passed" in out, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert res.returncode == 0, out[-3000:]
    shutil.rmtree(tmp_path / "obj", ignore_errors=True)
