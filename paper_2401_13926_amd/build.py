"""Builds libkkt.so (HIP kernels for gfx950 + host analysis + C ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import pathlib
import subprocess
import sys

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
LIB = PKG / "libkkt.so"
SOURCES = [PKG / "csrc" / "kkt_gpu.hip", PKG / "csrc" / "analysis.cpp", PKG / "csrc" / "server.cpp",
           PKG / "csrc" / "hykkt.hip"]
HEADERS = [PKG / "csrc" / "analysis.hpp", PKG / "csrc" / "kernels.hpp", ROOT / "include" / "kkt.h"]
ARCH = os.environ.get("KKT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def command(out: pathlib.Path) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", str(ROOT / "include"),
            "-o", str(out)] + [str(s) for s in SOURCES] + ["-lpthread"]


def build(force: bool = True) -> pathlib.Path:
    """Compile libkkt.so; with force=False only when a source is newer than the library."""
    if not force and LIB.exists():
        t = LIB.stat().st_mtime
        if all(p.stat().st_mtime <= t for p in SOURCES + HEADERS):
            return LIB
    tmp = LIB.with_name(LIB.name + ".tmp%d" % os.getpid())
    subprocess.run(command(tmp), check=True, cwd=str(PKG))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force="--if-stale" not in sys.argv)
    print(LIB)
