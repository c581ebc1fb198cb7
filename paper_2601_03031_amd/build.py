"""Build the gfx950 library (lib/libvc.so) and the host build of its arithmetic
(lib/libvc_hostcheck.so, used only by CPU tests).

    python -m paper_2601_03031_amd.build [--incremental] [-j N]

Kernel translation units compile in parallel with hipcc; packed FP32 instructions
are disabled on every HIP compile line.
"""
from __future__ import annotations

import argparse
import glob
import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(LIBDIR, "libvc.so")
HOSTCHECK = os.path.join(LIBDIR, "libvc_hostcheck.so")

UNITS = ["k_slp.hip", "k_verify.hip", "k_wide.hip", "k_g1.hip", "k_hash.hip", "vc.cpp"]
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + INCLUDE, "-I" + CSRC]


def _headers():
    return glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(CSRC, "*.h")) + [
        os.path.join(INCLUDE, "vc.h")]


def _stale(obj: str, src: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(p) > t for p in [src] + _headers())


def _compile(unit: str, incremental: bool, verbose: bool):
    src = os.path.join(CSRC, unit)
    obj = os.path.join(BUILD, unit + ".o")
    if incremental and not _stale(obj, src):
        return unit, 0.0, ""
    cmd = ["hipcc"] + HIPFLAGS + ["-c", src, "-o", obj + ".tmp"]
    if unit.endswith(".cpp"):
        cmd = ["hipcc", "-x", "hip"] + HIPFLAGS + ["-c", src, "-o", obj + ".tmp"]
    t0 = time.time()
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), p.stdout[-4000:], p.stderr[-4000:]))
    os.replace(obj + ".tmp", obj)
    return unit, time.time() - t0, " ".join(cmd) if verbose else ""


def generate() -> None:
    """Write the generated headers: curve constants and the engine's programs."""
    for script, out in (("gen_constants.py", "constants.hpp"), ("gen_slp.py", "slp_progs.hpp")):
        dst = os.path.join(CSRC, out)
        src = os.path.join(CSRC, script)
        if os.path.exists(dst) and os.path.getmtime(dst) >= os.path.getmtime(src):
            continue
        text = subprocess.run([sys.executable, src], capture_output=True, text=True, check=True).stdout
        with open(dst + ".tmp", "w") as f:
            f.write(text)
        os.replace(dst + ".tmp", dst)


def build(incremental: bool = False, verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    generate()
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(lambda u: _compile(u, incremental, verbose), UNITS))
    for unit, dt, cmd in results:
        if verbose:
            print("  %-12s %6.1f s  %s" % (unit, dt, cmd))
    objs = [os.path.join(BUILD, u + ".o") for u in UNITS]
    link = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    subprocess.run(link, check=True, capture_output=not verbose)
    os.replace(LIB + ".tmp", LIB)
    build_hostcheck()
    return LIB


def build_hostcheck() -> str:
    """Host (g++) build of the device arithmetic headers, with field-multiplication counters."""
    os.makedirs(LIBDIR, exist_ok=True)
    hc = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fvisibility=hidden", "-DVC_COUNT_MULS", "-I" + CSRC,
          "-o", HOSTCHECK + ".tmp", os.path.join(CSRC, "hostcheck.cpp")]
    subprocess.run(hc, check=True)
    os.replace(HOSTCHECK + ".tmp", HOSTCHECK)
    return HOSTCHECK


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("-j", type=int, default=8)
    a = ap.parse_args()
    t = time.time()
    build(incremental=a.incremental, verbose=True, jobs=a.j)
    print("built %s in %.1f s" % (LIB, time.time() - t))
    sys.exit(0)
