"""The reference stepper (oracle/btx_oracle.c) and libbtx's host-side grid
set-up (csrc/btx_grid.cpp) built with gcc's address and undefined-behaviour
sanitizers (host code only, no GPU code involved) and driven through every
grid kind and every entry point of the reference by tests/sanitize_driver.cpp.
Any out-of-bounds access, use after free, leak, signed overflow, misaligned
or null access aborts the driver with a report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="gcc/g++ not found")
def test_oracle_and_grid_under_asan_ubsan(tmp_path):
    objs = []
    for cc, std, src in (("gcc", "-std=c11", "oracle/btx_oracle.c"),
                         ("g++", "-std=c++17", "paper_2003_02845_amd/csrc/btx_grid.cpp"),
                         ("g++", "-std=c++17", "tests/sanitize_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([cc, std, "-ffp-contract=off"] + SAN + ["-c", os.path.join(ROOT, src), "-o", obj],
                       check=True, capture_output=True, text=True)
        objs.append(obj)
    exe = str(tmp_path / "sanitize_driver")
    subprocess.run(["g++"] + SAN + objs + ["-lm", "-o", exe], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(res.stdout)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "all cases done" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    assert res.stdout.count("zones,") == 6
