"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle and the library's host side (argument validation, overlap
checks, scheduling, layouts; no launches) are rebuilt instrumented, and the
oracle pins and the C-ABI tests run against those builds in a child process
with the sanitizer runtime preloaded.  Any report aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_tests(env, *files):
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join(ROOT, "tests", f) for f in files]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:] + r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_oracle_and_host_side_under_sanitizers(tmp_path):
    from oracle import build_oracle
    from paper_2311_07602_amd import build
    try:
        rt = build.sanitizer_runtime()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    orc = build_oracle.build_sanitized(str(tmp_path / "liblrbg_oracle_san.so"))
    try:
        lib = build.build_sanitized(str(tmp_path))
    except FileNotFoundError as e:
        pytest.skip(str(e))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", LRBG_ORACLE_LIB=orc, LRBG_LIB=lib)
    _run_tests(env, "test_oracle_pins.py", "test_abi.py", "test_svd_schedule.py")
