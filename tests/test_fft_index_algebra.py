"""Index algebra of the register-resident FFT passes, on the CPU.

The four-step split of the row and column passes (fft_reg.h) is host-callable;
tests/native/fft_reg_emu.cpp runs it for every thread of one workgroup, for
each (length, columns) and (length, threads per row) shape the library
instantiates, forward and inverse, and compares every line with a naive DFT.
No GPU is involved: this checks which thread computes which output before
any kernel runs.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "fft_reg_emu.cpp")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_register_fft_layouts_match_naive_dft(tmp_path):
    exe = str(tmp_path / "fft_emu")
    subprocess.run(["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", SRC, "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 2 * (7 + 9) and all("cover ok" in l for l in lines)
