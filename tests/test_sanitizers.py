"""The oracle and the library's host code built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only: the device code is compiled as usual and never runs here), each driven through its
C interface by a small program under `tests/sanitize/`. CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp"] + SAN +
                   ["-I" + os.path.join(ROOT, "oracle"), "-o", exe,
                    os.path.join(ROOT, "tests", "sanitize", "oracle_driver.cpp")], check=True)
    _run(exe)


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2608_15781_amd import build

    exe = str(tmp_path / "host_api_driver")
    host_san = []
    for flag in SAN:  # host pass only; the device code is built as usual
        host_san += ["-Xarch_host", flag]
    cmd = [build.hipcc(), "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san + [
        "-I" + os.path.join(ROOT, "include"), "-o", exe,
        os.path.join(ROOT, "tests", "sanitize", "host_api_driver.cpp")] + build.SOURCES
    subprocess.run(cmd, check=True, capture_output=True)
    _run(exe)
