"""The C-ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The translation units that validate arguments, carve workspaces and build
batch work lists are rebuilt with host-side ASan + UBSan (device code as
usual) and the CPU tests of the C-ABI (tests/test_abi.py: every rejection
path, workspace formulas, the allocation-free entry point's size check, the
injected allocation failure) run against that library in a fresh process
with the ASan runtime preloaded.  Any sanitizer report fails the test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2212_14318_amd import build as qbuild  # noqa: E402


def test_abi_checks_clean_under_asan_and_ubsan():
    rt = qbuild.asan_runtime()
    if rt is None or not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("clang ASan runtime or hipcc not available")
    try:
        lib = qbuild.build_host_sanitized()
    except RuntimeError as e:
        if "run build() first" in str(e):
            pytest.skip(str(e))
        raise
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "LD_LIBRARY_PATH": os.path.dirname(rt) + ":" + env.get("LD_LIBRARY_PATH", ""),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "QTPROD_LIB": lib,
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
