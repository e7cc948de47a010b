"""The tiled state layout, checked on the host: tests/layout_check.hip is built with hipcc
from the library's own header and run (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_tile_layout_is_a_bijection_with_contiguous_suffixes(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "layout_check"
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}",
           f"-I{os.path.join(ROOT, 'paper_2110_14934_amd', 'csrc')}", os.path.join(HERE, "layout_check.hip"),
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "layout ok" in r.stdout, r.stdout + r.stderr
