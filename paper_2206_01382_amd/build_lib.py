"""Compile libfpp.so (the HIP kernels and the C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfpp.so")

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = True, extra: list[str] | None = None, jobs: int | None = None) -> str:
    """Compile every source (in parallel) and link libfpp.so next to this file; returns its path."""
    import concurrent.futures
    import tempfile

    cc = hipcc()
    flags = [f for f in HIP_FLAGS if f != "-shared"] + (extra or [])
    objdir = tempfile.mkdtemp(prefix="fpp_build_")
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]

    def compile_one(pair):
        src, obj = pair
        cmd = [cc] + flags + ["-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l and "unknown target feature" not in l)
        return src, r.returncode, msg

    n = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    try:
        with concurrent.futures.ThreadPoolExecutor(max_workers=n) as ex:
            for src, rc, msg in ex.map(compile_one, zip(srcs, objs)):
                if msg.strip() and (verbose or rc):
                    print(msg, flush=True)
                if rc:
                    raise RuntimeError(f"hipcc failed on {src}")
        tmp = LIB + ".tmp"
        link = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
