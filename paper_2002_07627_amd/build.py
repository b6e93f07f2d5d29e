"""Build the HIP library libimf.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libimf.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["capi.cpp", "k_raster.hip", "k_fft.hip", "k_imf.hip", "k_couple.hip", "k_exact.hip"]
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# the rasterization predicate and the coupling arithmetic are evaluated exactly
# in the order written
# k_imf.hip and k_fft.hip never see a NaN (overlaps, minima and +inf padding
# only; a design holding one fails the request): without NaN semantics their
# minima and maxima need no input canonicalization
EXTRA = {"k_raster.hip": ["-ffp-contract=off"], "k_couple.hip": ["-ffp-contract=off"],
         "k_imf.hip": ["-fno-honor-nans"], "k_exact.hip": ["-ffp-contract=off"],
         "k_fft.hip": ["-fno-honor-nans"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc"] + COMMON + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, msg))
    if msg.strip():
        sys.stderr.write(msg + "\n")
    return obj


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
