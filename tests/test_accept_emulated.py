"""The accept kernel's lane logic, run on the CPU.

tests/emulated/ builds k_accept from the library's own source as host C++
(one thread per work-item, wavefront collectives as checked rendezvous) with
AddressSanitizer and UBSan, and drives it with random windows: replayed and
generated decisions, k_s = 16/32/64, windows with up to 64 elements, empty
and tiny orders, a removal or flip carried into the window, the order limit,
spin-flip proposals, removals and flips of one vertex in one window (closed
before the second touch, or rejected in the neglect mode).
It catches out-of-bounds accesses, collectives that some lanes skip
(divergence) and barriers not every wavefront reaches, and checks the
sweep algebra against determinant ratios of the Gram matrix and the
compaction plan against the surviving and inserted vertices and the flipped
auxiliary spins.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emulated")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_accept_kernel_emulated(tmp_path):
    hdr = tmp_path / "k_accept_emu.h"
    subprocess.run([sys.executable, os.path.join(EMU, "assemble.py"), ROOT, str(hdr)], check=True)
    exe = tmp_path / "accept_main"
    shutil.copy(os.path.join(EMU, "emu_hip.h"), tmp_path / "emu_hip.h")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I" + os.path.join(ROOT, "include"), "-I" + str(tmp_path),
                    os.path.join(EMU, "accept_main.cpp"), "-o", str(exe), "-lpthread"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe), "60"], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
