"""Build libih.so in-tree with hipcc for gfx950.

    python -m paper_1711_01919_amd.build        # or build() from Python

The library is placed next to this file so that a copy of the tree carries
it.  Compilation always runs (no staleness check), as the build check expects.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
LIB = PKG / "libih.so"
OBJDIR = PKG / "_build"

ARCH = os.environ.get("IH_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# Packed fp32 ops are switched off for all device code (none of the kernels
# here does floating point, but the flag keeps the compiler from ever emitting
# them).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          f"-I{INCLUDE}", f"-I{CSRC}"]

SOURCES = {
    "ih_kernels.hip": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_tile_regular.hip": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_tile_regular_guarded.hip": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_tile_nontemporal.hip": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_tile_nontemporal_guarded.hip": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_tile_table.hip": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_capi.cpp": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_batch.cpp": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_util.cpp": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_launch.cpp": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_server.cpp": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_pipeline.cpp": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_geom.cpp": ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS],
    "ih_admission.cpp": [],
}


def _compile(src: str, flags: list[str]) -> Path:
    obj = OBJDIR / (Path(src).stem + ".o")
    cmd = [HIPCC, *COMMON, *flags, "-c", str(CSRC / src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> Path:
    OBJDIR.mkdir(exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *map(str, objs), "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
