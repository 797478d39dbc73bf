"""Builds liblincoll.so for gfx950 in-tree with hipcc (no GPU needed).

    python -m paper_2503_09580_amd.build [--jobs N]

Each source compiles to an object in csrc/_build, then everything links into
paper_2503_09580_amd/_lib/liblincoll.so.  Always rebuilds.
"""
import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "liblincoll.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["abi.cpp", "host_tables.cpp", "staged.hip", "setup.hip", "fused.hip", "mfma_dft.hip", "timestep.hip", "quadcoll.hip", "steady.hip",
           "solver.cpp", "learn.hip", "mlp.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]
# packed FP32 instructions are kept out of every device code object
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fgpu-flush-denormals-to-zero"]


def compile_one(src):
    obj = os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON
    if src.endswith(".hip"):
        cmd += ["-x", "hip"] + DEVICE
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r.returncode, r.stdout + r.stderr


def build(jobs=4, verbose=False):
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_twiddles.py")], check=True)
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    os.makedirs(OUT_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = False
    for src, obj, rc, log in results:
        noisy = [l for l in log.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if rc != 0 or (verbose and noisy):
            print(f"--- {src} (rc={rc})\n" + "\n".join(noisy))
        failed |= rc != 0
    if failed:
        raise RuntimeError("compilation failed")
    objs = [r[1] for r in results]
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", LIB + ".tmp"] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        print(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose))
