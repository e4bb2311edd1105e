"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The sources are built a second time with the host pass instrumented (the
device code is unchanged) and the C ABI checks of test_abi.py run against
that build in a child process with the ASan runtime preloaded: argument
validation, configuration planning, workspace sizing and the batch and
checkpoint argument checks, with no GPU.  Any sanitizer report fails the
test (UBSan is built not to recover)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

CHILD = """
import sys
import paper_1211_5481_amd._lib as L
L.LIB_PATH = {lib!r}
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                      {tests!r}]))
"""


def test_abi_checks_clean_under_host_asan_and_ubsan():
    from paper_1211_5481_amd import build
    try:
        lib = build.build_sanitized(verbose=False)
        runtime = build.sanitizer_runtime()
    except RuntimeError as e:     # no ROCm toolchain here
        pytest.skip(f"sanitized build unavailable: {e}")
    env = dict(os.environ)
    # the ASan runtime must come first; anything already preloaded stays
    env["LD_PRELOAD"] = os.pathsep.join(x for x in (runtime, env.get("LD_PRELOAD", "")) if x)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    code = CHILD.format(lib=lib, tests=os.path.join(ROOT, "tests", "test_abi.py"))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout
