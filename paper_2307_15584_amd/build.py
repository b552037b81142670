"""Compile the HIP library libqmc.so for gfx950 in-tree (no JIT cache), and the VALU issue-rate
probe (valu_rate) that measures the instruction rates behind the per-pixel kernels' roofline.

  python -m paper_2307_15584_amd.build
"""

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
CSRC = os.path.join(PKG, "csrc")
BUILD_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqmc.so")
PROBE_SRC = os.path.join(CSRC, "probe", "valu_rate.cpp")
PROBE = os.path.join(PKG, "valu_rate")

SOURCES = ["context.hip", "setup.cpp", "generate.hip", "integrate.hip", "tune.hip"]

ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "--offload-arch=" + ARCH,
    # No packed-FP32 instructions: compile scalar FP32 code only.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _compile(src, verbose):
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc()] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compiling %s failed:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose=False, jobs=None):
    """Compile every source and link libqmc.so; returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), 8)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("linking libqmc.so failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


def build_probe(verbose=False):
    """The standalone VALU issue-rate probe (an executable, not part of the library)."""
    tmp = PROBE + ".tmp%d" % os.getpid()
    cmd = [_hipcc()] + [f for f in FLAGS if f != "-fPIC"] + ["-x", "hip", PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compiling valu_rate failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
