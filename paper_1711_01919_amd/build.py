"""Build libih.so in-tree for gfx950.

    python -m paper_1711_01919_amd.build        # or build() from Python

Kernel sources (.hip) are compiled by hipcc for gfx950; host-only sources
(.cpp) are plain C++ against the HIP runtime headers.  The library is placed
next to this file so that a copy of the tree carries it.  Compilation always
runs (no staleness check), as the build check expects.
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
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ROCM_INCLUDE = os.path.join(ROCM, "include")
ROCM_LIB = os.path.join(ROCM, "lib")

# Packed fp32 ops are switched off for all device code (none of the kernels
# here does floating point, but the flag keeps the compiler from ever emitting
# them).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          f"-I{INCLUDE}", f"-I{CSRC}"]
HIP = ["-x", "hip", f"--offload-arch={ARCH}", *DEVICE_FLAGS]
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM_INCLUDE}"]

# Sources holding kernels (device code), then host-only sources.
SOURCES = {
    "ih_kernels.hip": HIP,
    "ih_tile_regular.hip": HIP,
    "ih_tile_regular_guarded.hip": HIP,
    "ih_tile_nontemporal.hip": HIP,
    "ih_tile_nontemporal_guarded.hip": HIP,
    "ih_tile_table.hip": HIP,
    "ih_noalloc.hip": HIP,
    "ih_capi.cpp": HOST,
    "ih_batch.cpp": HOST,
    "ih_util.cpp": HOST,
    "ih_launch.cpp": HOST,
    "ih_server.cpp": HOST,
    "ih_pipeline.cpp": HOST,
    "ih_geom.cpp": HOST,
    "ih_admission.cpp": HOST,
}
HOST_SOURCES = [k for k, v in SOURCES.items() if v is HOST]

# Sanitizer builds for the CPU-only checks: the host-only sources compiled by
# the ROCm clang++ (plain C++, no offloading) with AddressSanitizer and UBSan,
# or with ThreadSanitizer, linked with the kernel objects of the regular build
# (which the sanitizers do not touch).  A process using such a library loads
# the matching clang runtime first (sanitizer_runtime()).
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
SANITIZE = {
    "address": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                "-shared-libasan"],
    "thread": ["-fsanitize=thread", "-fno-omit-frame-pointer"],
}


def sanitizer_runtime(kind: str) -> Path:
    """The clang runtime a process needs preloaded to use a sanitized build."""
    name = {"address": "libclang_rt.asan-x86_64.so", "thread": "libclang_rt.tsan-x86_64.so"}[kind]
    found = sorted(Path(ROCM, "llvm", "lib", "clang").glob(f"*/lib/linux/{name}"))
    if not found:
        raise FileNotFoundError(name)
    return found[-1]


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{what} failed:\n{' '.join(map(str, cmd))}\n{r.stdout}\n{r.stderr}")


def _compile(src: str, flags: list[str]) -> Path:
    obj = OBJDIR / (Path(src).stem + ".o")
    _run([HIPCC, *COMMON, *flags, "-c", str(CSRC / src), "-o", str(obj)], f"hipcc for {src}")
    return obj


def _compile_sanitized(src: str, kind: str, objdir: Path) -> Path:
    obj = objdir / (Path(src).stem + ".o")
    _run([CLANGXX, "-O1", "-g", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM_INCLUDE}",
          f"-I{INCLUDE}", f"-I{CSRC}", *SANITIZE[kind], "-c", str(CSRC / src), "-o", str(obj)],
         f"clang++ for {src}")
    return obj


def _link(objs, out: Path, tool: list[str]) -> Path:
    tmp = out.with_suffix(".so.tmp")
    _run([*tool, *map(str, objs), "-o", str(tmp)], "link")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> Path:
    OBJDIR.mkdir(exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    _link(objs, LIB, [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}"])
    if verbose:
        print(f"built {LIB}")
    return LIB


def build_sanitized(kind: str, out: Path) -> Path:
    """libih.so with its host-only sources under a sanitizer ("address": ASan
    and UBSan; "thread": TSan), at `out`.  The kernel objects come from the
    regular build (built first if missing)."""
    kernel_objs = [OBJDIR / (Path(src).stem + ".o") for src in SOURCES if src not in HOST_SOURCES]
    if not all(o.exists() for o in kernel_objs):
        build()
    out = Path(out)
    objdir = out.parent / f"_objs_{kind}"
    objdir.mkdir(parents=True, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        host_objs = list(ex.map(lambda src: _compile_sanitized(src, kind, objdir), HOST_SOURCES))
    return _link([*host_objs, *kernel_objs], out,
                 [CLANGXX, "-shared", "-fPIC", *SANITIZE[kind], f"-L{ROCM_LIB}", f"-Wl,-rpath,{ROCM_LIB}",
                  "-lamdhip64"])


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
