"""Build libslhjb.so (HIP kernels + C-ABI) in-tree for gfx950 with hipcc.

Run ``python -m paper_1502_01629_amd.build`` or call ``build()``.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libslhjb.so")
ARCH = "gfx950"

SOURCES = ["sweep.hip", "pipeline.hip", "tiles.hip", "batch.hip", "cnn.hip", "net.hip", "capi.hip"]

# -packed-fp32-ops: never emit packed FP32 VALU instructions (some of their forms have been
# seen to give wrong results on this hardware); hipcc's host pass warns that it does not
# know the feature, which is harmless.
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", f"-I{os.path.join(ROOT, 'include')}",
]


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of every source the library is built from: the HIP sources,
    the internal headers and the public header. Compiled into the library and checked on load."""
    h = hashlib.sha256()
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    for name in names:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "include", "slhjb.h"), "rb") as f:
        h.update(b"slhjb.h\0" + f.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    tag = source_hash()

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = [cc, *HIPCC_FLAGS, f'-DSLHJB_SOURCE_HASH="{tag}"', "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
