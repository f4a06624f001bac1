"""Compile libfs.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1702_07409_amd.build   (or build_library() from Python)
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfs.so")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-fvisibility=hidden",
          "-I" + INCLUDE, "-I" + CSRC]
# device code: no packed FP32 instructions (there is no float math in the
# kernels, the flag only keeps the compiler from emitting them)
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]

SOURCES = [
    ("kernels.hip", DEVICE),
    ("simdisk.hip", DEVICE),
    ("precode.hip", DEVICE),
    ("checks.hip", DEVICE),
    ("graph_dev.hip", DEVICE),
    ("api.cpp", DEVICE),
    ("plan.cpp", DEVICE),
    ("noalloc.cpp", DEVICE),
    ("graph_host.cpp", HOST),
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src, flags, cc):
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [cc, *flags, *COMMON, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return out


SYNTH_SRC = os.path.join(ROOT, "synth", "csrc", "datagen.hip")
SYNTH_LIB = os.path.join(ROOT, "synth", "libsynth.so")


def build_synth(verbose=False):
    """The seeded payload generator used by tests and the benchmark."""
    cc = hipcc()
    tmp = SYNTH_LIB + ".tmp"
    cmd = [cc, *DEVICE, "-O3", "-std=c++17", "-fPIC", "-shared", "-fvisibility=hidden", SYNTH_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, SYNTH_LIB)
    if verbose:
        print("built", SYNTH_LIB)
    return SYNTH_LIB


def build_library(verbose=False):
    """Compile every source and link libfs.so; returns the library path."""
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s[0], s[1], cc), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose=True)
    build_synth(verbose=True)
    sys.exit(0)
