"""Build liblbmrv.so (HIP, gfx950) in-tree.

Every .hip file under csrc/ is compiled separately (in parallel) and linked
into paper_1312_3297_amd/liblbmrv.so.  Always rebuilds; objects go to _build/.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build", "lbmrv")
LIB = os.path.join(PKG, "liblbmrv.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
    "-fconstexpr-steps=100000000", "-fexperimental-new-constant-interpreter",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(jobs=None, verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    # the heaviest translation units first
    srcs.sort(key=lambda s: (0 if "d3q27" in s else 1 if "d3q19" in s else 2, s))
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    # the bandwidth/counter calibration programs (not part of the library)
    for name in ("copy_bw", "stream_q"):
        cal = os.path.join(PKG, "calibrate", name + ".hip")
        exe = os.path.join(PKG, "calibrate", name)
        r = subprocess.run([HIPCC] + FLAGS + [cal, "-o", exe + ".tmp"], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("calibration build failed:\n%s\n%s" % (r.stdout, r.stderr))
        os.replace(exe + ".tmp", exe)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
