"""The FFT building blocks of the HIP kernels (csrc/fft.h) compiled for the
host with g++ (through a two-line stand-in for the HIP runtime header) and
checked against the DFT's definition summed in long double
(tests/fft_host_check.cpp): each transform at every length from 2 to 64,
forward and inverse, float and double, and the packing of two real sequences
into one complex transform.  Runs on the CPU; no HIP code is executed."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fft_building_blocks_match_the_dft(tmp_path):
    exe = str(tmp_path / "fft_host_check")
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-I", os.path.join(HERE, "hip_host_shim"),
           "-I", os.path.join(ROOT, "paper_2503_09580_amd", "csrc"), os.path.join(HERE, "fft_host_check.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "fft host check: ok" in r.stdout
