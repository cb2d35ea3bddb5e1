"""Build libwlcov.so in-tree with hipcc for gfx950.

Usage: python -m paper_1812_07437_amd.build   (or call build())
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libwlcov.so")
OBJ_DIR = os.path.join(HERE, "_build")

SOURCES = ["plan.cpp", "api.hip", "k_tables.hip", "k_gram.hip", "k_assemble.hip", "k_chol.hip", "k_update.hip",
           "k_lattice.hip", "k_chifact.hip", "k_woodbury.hip", "k_window.hip", "k_pca.hip", "server.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-function",
          "-Wno-unused-result"]
# Packed FP32 instructions are kept off for every device compilation.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ_DIR, src + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + DEVICE + COMMON + ["-c", path, "-o", obj]
    else:
        cmd = [HIPCC] + COMMON + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    # the host pass does not know the packed-fp32 feature; drop that harmless note
    noise = "is not a recognized feature for this target"
    msgs = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l).strip()
    return obj, msgs


def build(verbose=False):
    """Compile every HIP/C++ source for gfx950 and link libwlcov.so."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    for obj, msgs in results:
        if msgs and verbose:
            print(msgs, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
