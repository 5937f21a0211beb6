"""Build libddrom.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/model.hip", "csrc/kernels.hip", "csrc/mlp.hip", "csrc/aetrain.hip", "csrc/autotune.hip"]
OUT = os.path.join(HERE, "libddrom.so")


def hipcc_cmd(out=OUT, extra=()):
    return (["hipcc", "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]
            + list(extra) + [os.path.join(HERE, s) for s in SOURCES] + ["-o", out])


def build(verbose=True):
    tmp = OUT + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
