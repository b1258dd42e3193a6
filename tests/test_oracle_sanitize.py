"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_check.c calls every exported oracle function on small and
degenerate shapes with exactly sized buffers; built with gcc
-fsanitize=address,undefined and no recovery, any out-of-bounds access,
use of freed memory or undefined arithmetic ends the run with an error.  It
runs serially and with the OpenMP loops on 4 threads.  A copy of the oracle
with one planted write past the last product of a channel block must be
caught, so the harness is known to reach the accumulator bounds."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle", "oracle.c")
DRIVER = os.path.join(ROOT, "oracle", "sanitize_check.c")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


def build(tmp_path, name, src, openmp):
    exe = str(tmp_path / name)
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", *SAN, *(["-fopenmp"] if openmp else []),
           "-o", exe, src, DRIVER, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def run(exe, threads=1):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)


@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_runs_clean_under_asan_ubsan(tmp_path, openmp):
    exe = build(tmp_path, "osan", ORACLE, openmp)
    r = run(exe, threads=4 if openmp else 1)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "run clean" in r.stdout


def test_planted_overflow_is_caught(tmp_path):
    src = open(ORACLE).read()
    line = "                Vc[2 * b + 1] = im;\n"
    assert src.count(line) >= 1
    # one write past the last product of the channel block (first occurrence: the int8 X-engine)
    bad = src.replace(line, line + "                if (i == n_in - 1 && j == i) Vc[2 * b + 2] = 0;\n", 1)
    p = tmp_path / "oracle_bad.c"
    p.write_text(bad)
    exe = build(tmp_path, "osan_bad", str(p), False)
    r = run(exe)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
