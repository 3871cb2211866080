"""Builds libgee.so (hipcc, gfx950) in the package directory."""

from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libgee.so")
# GEE_DEBUG=1 build: the same library with the kernels' internal index checks compiled in
LIB_DEBUG = os.path.join(PKG, "libgee_debug.so")
SOURCES = ["gee_count.hip", "gee_csr.hip", "gee_embed.hip", "gee_bucket.hip", "gee_edge.hip", "gee_zsparse.hip", "gee_api.hip"]
ARCH = "gfx950"

# Packed fp32 VALU ops are kept off (hipcc still vectorizes scalar code without them).
HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build_library(out: str = LIB, verbose: bool = False, extra_flags=()) -> str:
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *extra_flags, "-shared", f"-I{INCLUDE}", f"-I{CSRC}", *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


def build_debug_library(verbose: bool = False) -> str:
    return build_library(LIB_DEBUG, verbose, extra_flags=("-DGEE_DEBUG=1",))


if __name__ == "__main__":
    print(build_library(verbose=True))
    print(build_debug_library(verbose=True))
