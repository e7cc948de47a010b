"""The short steps of the per-pixel body (fast_step, rank1_step) against the general step
(mix_step) on the GPU: for random mixtures and inputs, every pixel a short step takes must come
out bit for bit as the general step computes it, and rank1_step must take the pixels whose
rank-1 component matches and keeps its rank. The check program (tests/paths_check.hip) includes
the library's own device header and is built by the package's build step."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "paths_check")


def test_short_steps_bit_identical_to_the_general_step():
    assert os.path.exists(EXE), "tests/paths_check is built by __graft_entry__.build()"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0 and "paths ok" in r.stdout, r.stdout + r.stderr
