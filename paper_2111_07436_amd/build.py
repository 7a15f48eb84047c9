"""Build libcamp.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2111_07436_amd.build   (or call build())
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libcamp.so")
BUILD = os.path.join(PKG, "_build")

HIP_SOURCES = ["api.hip", "engine_wave.hip", "engine_wave_k64a.hip", "engine_wave_k64b.hip",
               "engine_wave_k64c.hip", "engine_wave_k128.hip", "engine_wave_k256.hip",
               "engine_lane.hip", "autotune.hip", "serve.hip", "noalloc.hip", "probe.hip"]
CXX_SOURCES = ["compile.cpp", "mech_json.cpp", "mech_pack.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
          "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-Wno-unused-value"]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {cmd[-1]}")
    return r.stderr


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append([hipcc, *COMMON, *HIP_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, s), "-o", o])
    for s in CXX_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append([hipcc, *COMMON, "-x", "c++", "-c", os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for w in ex.map(_run, jobs):
            if verbose and w:
                sys.stderr.write(w)
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
