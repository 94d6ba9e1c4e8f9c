"""Build the gfx950 shared library ``librelapack_mi355x.so`` next to this file.

One hipcc invocation over ``csrc/*.hip``. Flags:
  * ``--offload-arch=gfx950``: MI355X only;
  * ``-mllvm -amdgpu-mfma-vgpr-form``: matrix-core accumulators stay in
    ordinary VGPRs instead of being copied through AGPRs around every
    instruction;
  * ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32
    instructions are generated;
  * no fast-math: division and square root stay correctly rounded.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC_DIR = os.path.join(HERE, "csrc")
LIB_NAME = "librelapack_mi355x.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def sources():
    return sorted(glob.glob(os.path.join(SRC_DIR, "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link the shared library."""
    objs = []
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    # objects of sources that no longer exist are never linked; drop them
    live = {os.path.basename(src) + ".o" for src in sources()}
    for name in os.listdir(obj_dir):
        if name.endswith(".o") and name not in live:
            os.remove(os.path.join(obj_dir, name))
    procs = []
    for src in sources():
        obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], "-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "is not a recognized feature" not in ln]
        if p.returncode != 0 or verbose:
            sys.stderr.write("\n".join(lines) + "\n")
        if p.returncode != 0:
            failed = True
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB_PATH + ".tmp"
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp], check=True,
                   stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
