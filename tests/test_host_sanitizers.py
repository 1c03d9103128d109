"""The host-only part of the library (group closure and irreps, the QL
tridiagonal eigensolver, the FTLM and KPM thermal sums, their C entry points
and the host thread pool they use) built with g++ under the address and
undefined-behaviour sanitizers, and under the thread sanitizer; the host
library tests (tests/test_lib_host.py, minus the export check, which needs the
full library) run against each build in a child process with the sanitizer
runtime preloaded, and any finding fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

from conftest import ROOT

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++ and its sanitizer runtimes")


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_host_library_under_sanitizers(kind):
    from paper_2607_17429_amd import build
    so = build.build_host_sanitized(kind=kind)
    env = build.sanitizer_env(so, kind)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-s", "-p", "no:cacheprovider", "-p", "no:xdist",
                        os.path.join(ROOT, "tests", "test_lib_host.py"), "-k", "not exports"],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    report = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert marker not in r.stderr, report
    assert " passed" in r.stdout, report
