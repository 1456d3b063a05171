"""The host half of the library (selection, delay tables, beamforming plans: kk_host.cpp) built
with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only) and driven over the named
workload shapes, the eight window-class geometries, seeded random geometries and the error
paths (tests/sanitize/host_driver.cpp).  The driver also proves, pixel by pixel, that every
delay falls inside the record window its plan records: the bound the gather kernels' on-chip
window reads depend on."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
           os.path.join(ROOT, "paper_2603_22496_amd", "csrc", "kk_host.cpp"), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-5000:]
    assert "runtime error" not in r.stdout and "AddressSanitizer" not in r.stdout
    assert "0 failures" in r.stdout
