"""The CPU pins again, with the oracle built under AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, every finding fatal).

The pins check the oracle's values; this run checks that computing them reads
and writes only inside the caller's buffers and has no undefined behaviour
(shifts by 64, signed overflow, misaligned access), including the edge cases
the pins exercise: k = 32, s = k, m = k, H = 16, empty and short records, N
bases, 8- and 16-word shards.  The Python interpreter is not built with the
sanitizers, so their runtimes are preloaded into a child process.  No GPU.
"""

import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_stored_values.py", "tests/test_bench_counts.py"]


def _runtime(name):
    try:
        path = subprocess.run(["gcc", "-print-file-name=" + name], stdout=subprocess.PIPE, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_pins_pass_under_asan_and_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not found")
    oracle.build(force=True, sanitize=True)
    env = dict(os.environ)
    env.update({
        "SBF_ORACLE_SANITIZE": "1",
        "LD_PRELOAD": asan + ":" + ubsan,
        # the interpreter's own allocations are not the subject here
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS, cwd=ROOT,
                       env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=1200)
    tail = "\n".join(r.stdout.splitlines()[-40:])
    assert r.returncode == 0, tail
    assert "passed" in tail and "AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout, tail
