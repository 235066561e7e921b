"""The host-side set-up code (hostmath.cpp: grids, operators, weights, sigma,
eigen-decompositions, phi_1 factors) built with AddressSanitizer and
UndefinedBehaviorSanitizer for the CPU (g++, no device code) and run over
every coordinate at sizes 3 to 512."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_11558_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_setup_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "host_asan")
        cmd = ["g++", "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", CSRC,
               os.path.join(CSRC, "hostmath.cpp"), os.path.join(ROOT, "tests", "host_asan_driver.cpp"),
               "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        # a preloaded library, if the environment has one, stays in place: the
        # runtime is then told not to insist on coming first
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        print(r.stdout, r.stderr[-2000:])
        assert r.returncode == 0, r.stderr[-4000:]
        assert "host set-up ok" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
