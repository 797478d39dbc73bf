"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the plan precomputation (csrc/host_tables.cpp: quadrature, radial tables,
the phi_j octant, the hemisphere polar rule) compiled with g++ and the
sanitizers, driven over every supported size, both quadrature rules, node
counts from 1 to 2n and every hemisphere rule (tests/host_tables_sanitize.cpp).
No GPU and no HIP code involved."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_tables_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_tables_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(HERE, "host_tables_sanitize.cpp"),
           os.path.join(ROOT, "paper_2503_09580_amd", "csrc", "host_tables.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host tables: ok" in r.stdout
