"""CPU-only checks of the library's host code under sanitizers.

  - the serving loop's device-memory bookkeeping (ih_admission: first-fit
    arena, admission with eviction and retry, never-fits verdict, retention
    and readers) as a C++ unit test, under AddressSanitizer + UBSan and under
    ThreadSanitizer;
  - the serving loop's host paths through the C ABI from several threads
    (validation, budget rejection, queued work the scheduler fails on a
    machine without a usable device, latest-histogram queries, holds,
    statistics, polling, shutdown with queued work), against a build of
    libih.so whose host sources carry the sanitizer;
  - the Python-level CPU tests (ABI exports and argument checks, server
    validation) against the AddressSanitizer build;
  - the oracle's pin suite against an oracle built with AddressSanitizer and
    UBSan.

No kernel is launched: every path here stops before the device.  The
sanitized builds use the ROCm clang++ and its runtimes."""
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
CSRC = ROOT / "paper_1711_01919_amd" / "csrc"
CPP = Path(__file__).resolve().parent / "cpp"
sys.path.insert(0, str(ROOT))

from paper_1711_01919_amd import build as ihbuild  # noqa: E402

FLAGS = {"address": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-shared-libasan"],
         "thread": ["-fsanitize=thread"]}
ENV = {"address": {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "halt_on_error=1"},
       "thread": {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"}}


def run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env={**os.environ, **(env or {})}, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(map(str, cmd))} exited {r.returncode}\n{r.stdout[-4000:]}\n{r.stderr[-8000:]}"
    return r.stdout


def rt_dir(kind):
    return ihbuild.sanitizer_runtime(kind).parent


@pytest.fixture(scope="module")
def sanitized_libs(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitized")
    return {kind: ihbuild.build_sanitized(kind, d / kind / "libih.so") for kind in ("address", "thread")}


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_admission_unit(tmp_path, kind):
    exe = tmp_path / f"admission_{kind}"
    run([ihbuild.CLANGXX, "-std=c++17", "-O1", "-g", *FLAGS[kind], f"-I{CSRC}", str(CPP / "test_admission.cpp"),
         str(CSRC / "ih_admission.cpp"), "-o", str(exe), "-lpthread", f"-Wl,-rpath,{rt_dir(kind)}"])
    assert "admission tests passed" in run([str(exe)], ENV[kind])


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_server_host_paths(tmp_path, sanitized_libs, kind):
    lib = sanitized_libs[kind]
    exe = tmp_path / f"server_{kind}"
    run([ihbuild.CLANGXX, "-std=c++17", "-O1", "-g", *FLAGS[kind], f"-I{ROOT / 'include'}",
         str(CPP / "test_server_paths.cpp"), f"-L{lib.parent}", "-lih", f"-Wl,-rpath,{lib.parent}",
         f"-Wl,-rpath,{rt_dir(kind)}", "-o", str(exe), "-lpthread"])
    assert "server paths passed" in run([str(exe)], ENV[kind])


def test_python_cpu_tests_under_asan(sanitized_libs):
    env = {**ENV["address"], "LD_PRELOAD": str(ihbuild.sanitizer_runtime("address")),
           "IH_LIBRARY": str(sanitized_libs["address"])}
    out = run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
               str(ROOT / "tests" / "test_abi.py"), str(ROOT / "tests" / "test_server_cpu.py")], env)
    assert " passed" in out


def test_oracle_pins_under_asan(tmp_path):
    lib = tmp_path / "liboracle_asan.so"
    run(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", str(ROOT / "oracle" / "ih_oracle.c"), "-o", str(lib)])
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    script = ("import sys; sys.path[:0] = [%r, %r]\n"
              "import oracle\nfrom test_oracle_pins import pin_failures\n"
              "f = pin_failures(oracle.Oracle(%r))\nassert f == [], f\nprint('pins hold')\n"
              % (str(ROOT), str(ROOT / "tests"), str(lib)))
    out = run([sys.executable, "-c", script], {"LD_PRELOAD": libasan, "ASAN_OPTIONS": "detect_leaks=0",
                                               "UBSAN_OPTIONS": "halt_on_error=1"})
    assert "pins hold" in out
