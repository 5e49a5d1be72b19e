"""Builds libcloud.so (HIP for gfx950) in the package directory.

    python -m paper_1609_05344_amd.build

Every source is compiled with hipcc for gfx950 only; packed FP32 instructions
are disabled for all device code.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_NAME = "libcloud.so"
LIB_PATH = os.path.join(PKG, LIB_NAME)

SOURCES = ["render.hip", "taa.hip", "gather.hip", "composite.hip", "api.cpp", "serve.hip", "serve_core.cpp"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    return r


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source and link libcloud.so; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd.insert(1, "-xhip")
        objs.append(obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB_PATH + f".tmp{os.getpid()}"
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "lib")
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread",
          f"-L{rocm_lib}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{rocm_lib}"],
         verbose)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _wait(item):
    cmd, p = item
    out, err = p.communicate()
    if p.returncode != 0:
        sys.stderr.write(out + err)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    if err.strip():
        # hipcc's host pass warns about the device-only target feature; keep
        # everything else visible.
        lines = [l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
