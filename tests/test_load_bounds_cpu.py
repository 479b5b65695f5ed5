"""Regression guard for the kernels' global loads (CPU only, no GPU).

tests/load_bounds.hip calls the same __host__ __device__ address helpers the
kernels use (the strip, block-code and batch row loads, the in-place reads
of misaligned batch images, the histogram's chunk walk) for every lane position the kernels can
take: widths 1..2100, u8 and u16, aligned and misaligned bases and pitches,
rows past the image, several CU counts.  Every access must stay within a
16-byte block (aligned rows) or a dword (misaligned rows) that holds a pixel
of its own row.  A load that leaves its row can leave the allocation on the
last row, which faults the GPU, so a change to these helpers that breaks the
rule fails here first.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not installed")
def test_every_load_stays_in_its_row(tmp_path):
    exe = str(tmp_path / "load_bounds")
    src = os.path.join(ROOT, "tests", "load_bounds.hip")
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1710_06189_amd", "csrc"),
           src, "-o", exe]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 outside their row" in r.stdout
