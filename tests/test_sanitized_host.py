"""The host logic of the C-ABI library (FD weights, own eigensolver, scalar matrix functions,
plan-free helpers) under AddressSanitizer and UndefinedBehaviorSanitizer: tests/test_abi_cpu.py
runs in a subprocess against the host-sanitizer build (`python -m paper_2510_21394_amd.build
--sanitize`), with clang's ASan runtime preloaded.  CPU only; skipped when that build is absent
(it is not part of the default build)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_LIB = os.path.join(ROOT, "paper_2510_21394_amd", "_build_san", "libfcgle_san.so")


@pytest.mark.skipif(not os.path.exists(SAN_LIB), reason="host-sanitizer build not present")
def test_abi_cpu_under_asan_and_ubsan():
    from paper_2510_21394_amd.build import asan_runtime
    env = dict(os.environ, LD_PRELOAD=asan_runtime(), FCGLE_LIB=SAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
