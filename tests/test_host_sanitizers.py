"""The host library under AddressSanitizer and UndefinedBehaviorSanitizer, on
the CPU.

Every source of the library is compiled for the host only (no device code:
an empty GPU binary is embedded, so kernel launches become plain host calls)
with the sanitizers on, and linked with ``hip_host_stub.cpp`` (a host-memory
stand-in for the HIP runtime calls the library makes: exact-size allocations,
immediate copies, launch shapes checked and counted) and ``abi_driver.c``, a C
program that calls every entry point of ``include/lbrd.h`` on tiny and ragged
lattices, batches and the server, including the error paths.  Any
out-of-bounds access of a staging copy, descriptor upload or arena slot, any
use after free, leak or undefined operation in the host code fails the run.
Kernels run nothing here; the numbers are checked by the same driver on a GPU
(``test_gpu_abi_driver.py``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1007_3109_amd" / "csrc"
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]
SAN_PLAIN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(" ".join(map(str, cmd)) + "\n" + r.stderr[-4000:])


@pytest.mark.skipif(not (Path(HIPCC).exists() and Path(CLANGXX).exists()), reason="ROCm compilers not available")
def test_host_library_clean_under_sanitizers(tmp_path):
    empty = tmp_path / "empty_gpu_binary"
    empty.write_bytes(b"")
    common = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC", f"-I{ROOT / 'include'}", f"-I{CSRC}"]
    sources = sorted(list(CSRC.glob("*.hip")) + list(CSRC.glob("*.cpp")))

    def compile_one(src):
        obj = tmp_path / (src.name + ".o")
        _run([HIPCC, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-Xclang", "-fcuda-include-gpubinary",
              "-Xclang", str(empty), *common, *SAN, "-c", str(src), "-o", str(obj)])
        return str(obj)

    with ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, sources))
    stub = tmp_path / "stub.o"
    _run([CLANGXX, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-O1", "-g", "-std=c++17", *SAN_PLAIN, "-c",
          str(ROOT / "tests" / "hip_host_stub.cpp"), "-o", str(stub)])
    drv = tmp_path / "driver.o"
    _run([CLANG, "-O1", "-g", "-std=c11", f"-I{ROOT / 'include'}", *SAN_PLAIN, "-c",
          str(ROOT / "tests" / "abi_driver.c"), "-o", str(drv)])
    exe = tmp_path / "abi_driver"
    _run([CLANGXX, *SAN_PLAIN, str(drv), str(stub), *objs, "-o", str(exe), "-lpthread", "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe), "stub"], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "0 failures" in r.stdout, out[-6000:]
