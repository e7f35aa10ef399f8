"""Builds libmelt.so (HIP C++ for gfx950) in-tree with hipcc.

    python -m paper_2606_01009_amd.build      # or: from paper_2606_01009_amd.build import build

Every source under csrc/ is compiled to an object (in parallel) and linked into
paper_2606_01009_amd/_lib/libmelt.so.  Packed-FP32 instructions are disabled for the device
code; the host pass warns that it does not know that target feature, which is harmless.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
OUT_DIR = PKG / "_lib"
LIB = OUT_DIR / "libmelt.so"
ARCH = os.environ.get("MELT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", str(PKG.parent / "include"), "-I", str(CSRC)]


def build(verbose: bool = False, jobs: int | None = None) -> Path:
    """Compile every csrc source and link libmelt.so.  Always rebuilds."""
    OUT_DIR.mkdir(exist_ok=True)
    obj_dir = OUT_DIR / "obj"
    if obj_dir.exists():
        shutil.rmtree(obj_dir)          # objects of removed sources must not link
    obj_dir.mkdir()
    srcs = sorted([p for p in CSRC.iterdir() if p.suffix in (".hip", ".cpp")])
    cc = hipcc()

    def compile_one(src: Path) -> Path:
        obj = obj_dir / (src.name + ".o")
        cmd = [cc, *_flags(), "-c", str(src), "-o", str(obj)]
        if src.suffix == ".cpp":
            cmd[1:1] = ["-x", "hip"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src.name}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    n = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
