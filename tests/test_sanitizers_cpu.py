"""Host sanitizer runs: the library's host C++ (preprocessing, codebook
generation, checksummed file IO) and the C oracle, each built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, -fno-sanitize-recover)
into a driver program under tests/sanitize/ that exercises every entry point
with ragged and edge-case inputs. A sanitizer report or a failed invariant
makes the program exit non-zero. Device code is not covered (no GPU
sanitizer on this hardware)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2211_16422_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-ffp-contract=off"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(cmd, exe):
    if shutil.which(cmd[0]) is None:
        pytest.skip(f"{cmd[0]} not found")
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr + b.stdout).lower():
        pytest.skip("sanitizer runtime unavailable: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    out = _build_and_run(
        ["g++", "-std=c++17", *SAN, f"-I{CSRC}", os.path.join(HERE, "sanitize", "host_sanitize.cpp"),
         os.path.join(CSRC, "preprocess.cpp"), os.path.join(CSRC, "codebook.cpp"),
         os.path.join(CSRC, "persist.cpp"), "-o", exe, "-lpthread"], exe)
    assert "all checks passed" in out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    out = _build_and_run(
        ["gcc", "-std=c11", *SAN, "-mpopcnt", os.path.join(HERE, "sanitize", "oracle_sanitize.c"),
         os.path.join(ROOT, "oracle", "hyperoms_oracle.c"), "-o", exe, "-lm"], exe)
    assert "all checks passed" in out
