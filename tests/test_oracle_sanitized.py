"""The oracle's pins again, with the oracle built under AddressSanitizer and UndefinedBehaviorSanitizer.

The FP64 oracle is the reference for every parity check, so undefined behaviour in it (a signed
overflow, an out-of-bounds read) would make its answers depend on the compiler. This test builds a
separate instrumented copy of the oracle (-fsanitize=address,undefined, -fno-sanitize-recover=all),
runs every oracle pin file in a child process that preloads the sanitizer runtimes and stops at the
first report, and fails on a non-zero exit or any sanitizer report in the output. CPU only.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ("test_oracle_pins.py", "test_oracle_prune.py", "test_oracle_compact.py", "test_oracle_sh.py",
             "test_oracle_train.py")


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_clean_under_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc's sanitizer runtimes are not installed")
    env = dict(os.environ)
    env.update({
        "MEGS_ORACLE_SANITIZE": "1",
        "LD_PRELOAD": f"{asan}:{ubsan}",
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    files = [os.path.join(ROOT, "tests", f) for f in PIN_FILES]
    r = subprocess.run([sys.executable, "-m", "pytest", *files, "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    for marker in ("runtime error:", "ERROR: AddressSanitizer", "ERROR: LeakSanitizer"):
        assert marker not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out and " failed" not in out, out[-2000:]
