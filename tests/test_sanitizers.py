"""The host-side code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the C oracle built with clang's sanitizers, the library's host
code (validation, layout, planner, argument checks, the two-level
minimiser, Simplify) built with host-only sanitizer flags, and the host
tests run against both in a child process with the sanitizer runtime
preloaded.  Any report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RUNTIME = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))


@pytest.mark.skipif(not RUNTIME, reason="clang sanitizer runtime not installed")
def test_host_code_under_asan_and_ubsan():
    import oracle
    from paper_2502_08673_amd import build as b

    libtt = b.build(sanitize=True)
    liboracle = oracle.build(force=True, sanitize=True)
    env = dict(os.environ)
    env.update(LD_PRELOAD=RUNTIME[-1], TT_LIBRARY=libtt, ORACLE_LIBRARY=liboracle,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = ["tests/test_abi_host.py", "tests/test_sop_host.py", "tests/test_oracle_pins.py",
             "tests/test_oracle_sop.py", "tests/test_oracle_transform.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, out
    assert " passed" in r.stdout, out
