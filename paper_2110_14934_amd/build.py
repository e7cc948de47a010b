"""Build step of the HIP library: compiles every source under csrc/ for gfx950 with hipcc and
links them into ``libgmm.so`` next to this file (in-tree, so it travels with the package)."""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(HERE, "libgmm.so")

ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off; plain fp32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fp32 denormals are kept (IEEE behaviour); fused multiply-add is allowed except where a
    # "#pragma clang fp contract(off)" asks for separately rounded products and sums
    "-fno-gpu-flush-denormals-to-zero", "-ffp-contract=fast-honor-pragmas",
    # the per-pixel mixture must live in registers. The vector-combine pass widens a scalar read
    # of a mixture field (in a helper optimised before it is inlined) into a 16-byte vector
    # read; after inlining that read spans several fields, the mixture can no longer be split
    # into registers and the backend moves it to LDS (~7-20 KB per block, an LDS round trip
    # per access). Without the pass every frame kernel keeps only its 768-byte RGB staging.
    "-mllvm", "-disable-vector-combine",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [hipcc(), *HIP_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


# Device-code checks that the GPU tests run: built with the library's flags, in-tree, next to
# their sources (tests/<name>.hip -> tests/<name>).
CHECKS = [os.path.join(ROOT, "tests", "paths_check.hip")]


def check_path(src: str) -> str:
    return os.path.splitext(src)[0]


def _compile_check(src: str) -> str:
    exe = check_path(src)
    cmd = [hipcc(), *HIP_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", src, "-o", exe + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    os.replace(exe + ".tmp", exe)
    return exe


def build(verbose: bool = False) -> str:
    """Compile and link the library and the device-code checks; always rebuilds. Returns the
    library path."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    checks = [c for c in CHECKS if os.path.exists(c)]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs) + len(checks))) as ex:
        check_jobs = [ex.submit(_compile_check, c) for c in checks]
        objs = list(ex.map(_compile, srcs))
        for j in check_jobs:
            j.result()
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
