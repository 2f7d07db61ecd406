"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Two drivers, each built with g++ -fsanitize=address,undefined and run as its
own executable (no instrumented library is loaded into Python):

* tests/sanitize/sanitize_oracle.cpp with the oracle (oracle/dwos_oracle.cpp):
  forward and differential walks in 2D and 3D, walks on stars with a Robin
  condition and wall starts, an implicit boundary, the network;
* tests/sanitize/sanitize_host.cpp with the library's host sources
  (paper_2405_12964_amd/csrc/bvh_build.cpp and remesh.cpp): BVH builds on a
  sphere, a triangle soup and a polyline, remeshing and its error path.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-pthread"]


def _build_and_run(tmp_path, name, sources, extra=()):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    subprocess.run(["g++", *SAN, *extra, "-o", exe, *sources], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert f"{name}: ok" in out, out[-2000:]


def test_oracle_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "sanitize_oracle", [os.path.join(ROOT, "tests", "sanitize", "sanitize_oracle.cpp")])


def test_host_library_code_under_sanitizers(tmp_path):
    if not os.path.isdir("/opt/rocm/include/hip"):
        pytest.skip("HIP headers not available")
    csrc = os.path.join(ROOT, "paper_2405_12964_amd", "csrc")
    _build_and_run(tmp_path, "sanitize_host",
                   [os.path.join(ROOT, "tests", "sanitize", "sanitize_host.cpp"),
                    os.path.join(csrc, "bvh_build.cpp"), os.path.join(csrc, "remesh.cpp")],
                   extra=("-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"))
