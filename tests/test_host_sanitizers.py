"""The library's host C++ (table builders, partial-wave sums, photodissociation
spectra) built with AddressSanitizer and UndefinedBehaviorSanitizer and run by
tests/sanitize/host_driver.cpp: any out-of-bounds access, leak or undefined
behaviour aborts the driver.  CPU only (g++)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_10167_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
           os.path.join(CSRC, "host_tables.cpp"), os.path.join(CSRC, "partial_waves.cpp"),
           os.path.join(CSRC, "spectra.cpp")]


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory(prefix="tdwp_san_") as tmp:
        exe = os.path.join(tmp, "host_driver")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread",
               *SOURCES, "-o", exe]
        res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
        assert res.returncode == 0, res.stderr[-4000:]
        # the environment is passed as it is; ASan is told not to insist on coming
        # first among the loaded libraries
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
        assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
        assert "all checks passed" in run.stdout
