"""The host code of the HIP library (argument checks, prefactors, launch
logic, the host copy of the pixel ordering) and the oracle, built with
AddressSanitizer and UndefinedBehaviorSanitizer, under the CPU test suite.

The sanitized builds are separate files (libsynmarch_san.so,
libsync_oracle_san.so); a child pytest loads them in place of the normal ones
(SYNMARCH_LIB, SYNC_ORACLE_LIB) with the clang ASan runtime preloaded, and
any report (ASan aborts, UBSan halts on the first error) fails the run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_cpu_suite_under_asan_and_ubsan():
    from paper_2410_01136_amd import _build
    import oracle
    lib = _build.build(sanitize=True)
    olib = oracle.build(sanitize=True)
    env = dict(os.environ)
    env.update(LD_PRELOAD=_build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               SYNMARCH_LIB=lib, SYNC_ORACLE_LIB=olib, PYTHONDONTWRITEBYTECODE="1")
    # the sanitized files are the ones a child process loads
    probe = ("import oracle, paper_2410_01136_amd.binding as b; oracle._load(); "
             "m = open('/proc/self/maps').read(); "
             "print(int('libsynmarch_san.so' in m), int('libsync_oracle_san.so' in m), "
             "int('libclang_rt.asan' in m))")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == ["1", "1", "1"], r.stdout
    r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-q", "-x", "-m", "not gpu and not slow",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in r.stdout
