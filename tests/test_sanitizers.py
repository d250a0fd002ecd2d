"""Host code under AddressSanitizer and UBSan on the CPU: the oracle's
SymDel routes against its own brute-force routes (tests/sanitize/
oracle_checks.cpp), and the library's host staging (csrc/stage.cpp) with
host memory standing in for the device (tests/sanitize/stage_checks.cpp).
Each is built with g++ into a temporary folder and must print "ok"."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-pthread"]


def build_and_run(tmp_path, name, sources, extra=()):
    exe = str(tmp_path / name)
    subprocess.run(["g++", *SAN, *extra, *sources, "-o", exe], check=True, cwd=str(tmp_path),
                   timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    print(r.stderr)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_sanitizers(tmp_path):
    build_and_run(tmp_path, "oracle_checks",
                  [os.path.join(ROOT, "oracle", "symdel_oracle.cpp"),
                   os.path.join(ROOT, "tests", "sanitize", "oracle_checks.cpp")])


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_host_staging_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2403_09010_amd", "csrc")
    build_and_run(tmp_path, "stage_checks",
                  [os.path.join(csrc, "stage.cpp"),
                   os.path.join(ROOT, "tests", "sanitize", "stage_checks.cpp")],
                  ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                   "-I" + os.path.join(ROOT, "include"), "-I" + csrc])
