"""The host SELL-64 layout builder (csrc/afc_layout.cpp) under AddressSanitizer
and UndefinedBehaviorSanitizer: random CSR patterns, including bands wide
enough for 32-bit deltas, empty rows and rows without a diagonal, laid out and
checked entry by entry (tests/fuzz_sell_layout.cpp).  Host code only, built
with g++."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_layout_builder_is_clean_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "fuzz_sell_layout")
    cmd = ["g++", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-std=c++17",
           "-I", os.path.join(ROOT, "paper_2110_15676_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "fuzz_sell_layout.cpp"),
           os.path.join(ROOT, "paper_2110_15676_amd", "csrc", "afc_layout.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr or "").lower():
        pytest.skip("sanitizer runtime not available")
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "400", "300", "40000", "20"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout
