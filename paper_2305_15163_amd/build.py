"""Build libddrom.so in-tree with hipcc for gfx950.

Each source is compiled to an object of its own (in parallel), then the objects are
linked into the shared library.  Kernels are launched only from the file that defines
them, so no relocatable device code is needed."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/model.hip", "csrc/kernels.hip", "csrc/mlp.hip", "csrc/aetrain.hip", "csrc/autotune.hip"]
OUT = os.path.join(HERE, "libddrom.so")
OBJDIR = os.path.join(HERE, "_build")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _includes():
    return ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def _compile(src, extra, verbose):
    obj = os.path.join(OBJDIR, os.path.basename(src).replace(".hip", ".o"))
    cmd = ["hipcc"] + FLAGS + _includes() + list(extra) + ["-c", os.path.join(HERE, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    return obj, res


def build(verbose=True, extra=(), out=OUT):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, extra, verbose), SOURCES))
    bad = [r for _, r in results if r.returncode != 0]
    for _, r in results:
        if r.returncode != 0 or (verbose and r.stderr.strip()):
            sys.stderr.write(r.stdout + r.stderr)
    if bad:
        raise RuntimeError("hipcc failed")
    tmp = out + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950"] + [o for o, _ in results] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
