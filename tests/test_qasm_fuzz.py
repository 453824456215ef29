"""The circuit front end (host code) under AddressSanitizer and
UndefinedBehaviorSanitizer: random mutations of valid OpenQASM programs are
parsed and fused; every input must be accepted or rejected cleanly, and
fusion must never grow a circuit."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++ for the sanitizer build")
def test_parser_and_fusion_under_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "fuzz_qasm")
        subprocess.check_call(
            ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
             "-I", os.path.join(ROOT, "include"), "-o", exe,
             os.path.join(ROOT, "tests", "fuzz_qasm.cpp"),
             os.path.join(ROOT, "paper_2601_04422_amd", "csrc", "tnsim_qasm.cpp")])
        r = subprocess.run([exe, "30000"], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
        ok = int(r.stdout.split()[1])
        assert ok > 100  # some mutated programs stay valid and reach fusion
