"""libcorr's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/bin/host_sanitize_check (built by tests/hostcheck.py, which
__graft_entry__.build() calls) links the library's host sources compiled
with -fsanitize=address,undefined (host side only) to a driver that walks
every entry point's argument checks, configuration validation and workspace
sizing over a grid of valid and invalid configurations, and plan creation,
dump sizing and destruction.  Without a GPU the launches fail cleanly and the
plan's error state is exercised; on the GPU the driver also runs a small
integration through a plan and through the serving scheduler (its threads,
pinned completion words and persistent grid) and compares the sums with a
direct host sum.  Any memory error or undefined behaviour ends the run."""
import os
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import hostcheck  # noqa: E402


def run(args, leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={1 if leaks else 0}", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([hostcheck.EXE, *args], capture_output=True, text=True, env=env, timeout=300)


def test_host_library_clean_without_gpu():
    hostcheck.build()
    r = run([], leaks=True)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "run clean" in r.stdout


@pytest.mark.gpu
def test_host_library_clean_on_gpu():
    if not os.path.exists(hostcheck.EXE):
        pytest.skip("tests/bin/host_sanitize_check is built by __graft_entry__.build()")
    print("[host sanitizer] plan and scheduler paths on the GPU", flush=True)
    r = run(["gpu"], leaks=False)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "with GPU paths" in r.stdout
