"""The oracle's CPU tests again, with the oracle built under AddressSanitizer
and UndefinedBehaviorSanitizer (host code only): any out-of-bounds access,
use after free or undefined operation in the oracle fails this test."""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_tests_clean_under_asan_ubsan():
    from oracle import build
    lib = build.build(sanitize=True)
    env = dict(os.environ)
    env.update({"QOZ_REF_LIB": lib,
                "LD_PRELOAD": build.sanitizer_runtime(),
                # the interpreter's own allocations are not the oracle's
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    assert files
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x",
                        "-p", "no:cacheprovider", "-m", "not gpu"] + files,
                       cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout + r.stderr
    assert "runtime error" not in out, out[-4000:]
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
