"""The host-only ABI tests against a build of the library whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer (paper_2411_00033_amd/sanitize.py; the
device code is built as in the product and never runs here).  The tests run in a child
process with the ASan runtime preloaded; any report fails them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_tests_under_asan_and_ubsan():
    from paper_2411_00033_amd import sanitize
    rt = sanitize.runtime()
    if not rt:
        pytest.skip("no ASan runtime next to hipcc's clang")
    lib = sanitize.build() if sanitize.stale() else sanitize.LIB
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    code = ("import sys, pytest; sys.path.insert(0, %r); sys.path.insert(0, %r); "
            "from paper_2411_00033_amd import _lib; _lib.LIB_PATH = %r; "
            "sys.exit(pytest.main(['-q', '-m', 'not gpu', '-p', 'no:cacheprovider', %r]))"
            % (ROOT, os.path.join(ROOT, "tests"), lib, os.path.join(ROOT, "tests", "test_abi_host.py")))
    res = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, stdout=subprocess.PIPE,
                         stderr=subprocess.STDOUT, text=True, timeout=600)
    assert res.returncode == 0, res.stdout[-4000:]
    assert "ERROR: AddressSanitizer" not in res.stdout and "runtime error:" not in res.stdout, res.stdout[-4000:]
