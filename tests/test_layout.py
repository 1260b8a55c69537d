"""CPU check of the MFMA slice layout shared by the covariance build and
the FP32 scan (compiled host-only from the library's own header)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_fragment_pairs_cover_the_triangle_once(tmp_path):
    exe = tmp_path / "layout_check"
    cmd = ["/opt/rocm/bin/hipcc", "-std=c++17", "-O1", "--offload-arch=gfx950", "-x", "hip",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2002_07858_amd", "csrc"),
           os.path.join(HERE, "layout_check.cpp"), "-o", str(exe)]
    if not os.path.exists(cmd[0]):
        pytest.skip("hipcc not available")
    subprocess.check_call(cmd)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    assert out.strip().endswith("ok"), out
    # 4-row slices issued per 64 universes: 2 ns (ns+1) - P ns
    assert "N=57: 435" in out and "N=38: 200" in out and "N=64: 544" in out
