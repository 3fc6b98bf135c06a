"""The C ABI tests against a build whose host code runs under AddressSanitizer
and UndefinedBehaviorSanitizer (CPU only): argument checks, error paths and
the no-device path of every entry point the ABI tests reach, with any
invalid memory access or undefined behaviour in the library's host code
ending the run."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_pass_under_host_sanitizers():
    from paper_1912_03174_amd import build as B
    lib = B.build(verbose=False, sanitize=True)
    env = dict(os.environ, TDDFTB_LIB=lib, LD_PRELOAD=B.sanitizer_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", "tests/test_abi.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in out
    assert "runtime error" not in out                 # UndefinedBehaviorSanitizer
