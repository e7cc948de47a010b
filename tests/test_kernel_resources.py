"""Every kernel of the library keeps its per-pixel mixture in registers: compiled for gfx950
with the library's own flags, no kernel uses private (scratch) memory. A layout object or a
mixture array that the compiler cannot break into registers lands in scratch and costs a memory
round trip per access (a kernel that did so ran three times slower), so this is checked on the
host at build time."""
import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2110_14934_amd import build as B


def _resources(src):
    cmd = [B.hipcc(), *B.HIP_FLAGS, f"-I{B.INCLUDE}", f"-I{B.CSRC}", "-c", src, "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage", "--cuda-device-only"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            out[name] = int(m.group(1))
    return out


def test_no_kernel_uses_scratch():
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    with ThreadPoolExecutor(max_workers=min(8, len(B.sources()))) as ex:
        results = list(ex.map(_resources, B.sources()))
    kernels = {k: v for r in results for k, v in r.items()}
    assert any("batch_kernel" in k for k in kernels) and any("frame_kernel" in k for k in kernels)
    bad = {k: v for k, v in kernels.items() if v}
    assert not bad, bad
