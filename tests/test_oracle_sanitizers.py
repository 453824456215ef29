"""The CPU oracle under sanitizers (host builds only): AddressSanitizer with
UndefinedBehaviorSanitizer, and ThreadSanitizer over its OpenMP loops (the
rounds of the Jacobi SVD and the shots of the sampler).  The driver
tests/oracle_sanitize.c calls every entry point on seeded inputs.  A copy of
the oracle with a planted data race checks that the ThreadSanitizer build
does see races in these loops."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle", "tnsim_oracle.c")
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitize.c")
CLANG = "/opt/rocm/llvm/bin/clang"
LLVM_LIB = "/opt/rocm/llvm/lib"
ARCHER = os.path.join(LLVM_LIB, "libarcher.so")
have_tsan = os.path.exists(CLANG) and os.path.exists(ARCHER)


def _run(exe, env=None):
    return subprocess.run([exe], capture_output=True, text=True, timeout=600,
                          env=dict(os.environ, **(env or {})))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_asan")
        subprocess.check_call(
            ["gcc", "-std=gnu99", "-O1", "-g", "-fcx-fortran-rules", "-fopenmp",
             "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             "-fno-sanitize-recover=all", "-o", exe, DRIVER, ORACLE, "-lm"])
        r = _run(exe, {"OMP_NUM_THREADS": "4"})
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.strip().endswith("done")
        assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr


def _tsan_build(src, exe):
    subprocess.check_call(
        [CLANG, "-std=gnu99", "-O1", "-g", "-fcx-fortran-rules", "-fopenmp",
         "-fsanitize=thread", "-o", exe, DRIVER, src, "-lm", f"-Wl,-rpath,{LLVM_LIB}"])


TSAN_ENV = {"OMP_NUM_THREADS": "4", "OMP_TOOL_LIBRARIES": ARCHER,
            # the OpenMP runtime itself is not instrumented; archer supplies
            # its synchronisation to the sanitizer
            "TSAN_OPTIONS": "halt_on_error=1 ignore_noninstrumented_modules=1"}


@pytest.mark.skipif(not have_tsan, reason="needs clang with the OpenMP archer tool")
def test_oracle_under_thread_sanitizer():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_tsan")
        _tsan_build(ORACLE, exe)
        r = _run(exe, TSAN_ENV)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.strip().endswith("done")
        assert "data race" not in r.stderr


@pytest.mark.skipif(not have_tsan, reason="needs clang with the OpenMP archer tool")
def test_thread_sanitizer_sees_a_planted_race():
    src = open(ORACLE).read()
    planted = src.replace("reduction(| : rotated) ", "")
    assert planted != src
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "oracle_race.c")
        open(path, "w").write(planted)
        exe = os.path.join(tmp, "oracle_race")
        _tsan_build(path, exe)
        r = _run(exe, TSAN_ENV)
        assert r.returncode != 0 and "data race" in r.stderr
