"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): every decoder on small inputs, no invalid access, leak or UB."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitize")
        subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               os.path.join(ROOT, "oracle", "ngdbf_oracle.c"),
                               os.path.join(HERE, "c", "oracle_sanitize_main.c"),
                               "-lm", "-pthread", "-o", exe])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                           env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.strip() == "ok"
