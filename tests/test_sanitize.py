"""Host sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer, no recovery): the CPU
oracle built with gcc, and the library's host-only logic (planning, workspace query, option
validation, error strings) built with hipcc with the sanitizers on the host side only
(-Xarch_host), each driven by a small C/C++ program under tests/sanitize/.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "clean" in out.stdout
    return out.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-g"] + SAN + ["-o", exe, os.path.join(HERE, "oracle_main.c"),
                                                        os.path.join(ROOT, "oracle", "tikh_oracle.c"), "-lm",
                                                        "-fopenmp"])
    _run(exe)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_driver_host_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "driver_san")
    host = []
    for f in SAN:
        host += ["-Xarch_host", f]
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950"] + host +
                          ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
                           "-o", exe, os.path.join(HERE, "driver_host_main.cpp"),
                           os.path.join(ROOT, "paper_1302_6945_amd", "csrc", "tikh_driver.hip")],
                          stderr=subprocess.DEVNULL)
    _run(exe)
