"""A C program drives liblbrd.so through include/lbrd.h alone, on the GPU.

``abi_driver.c`` (the same program the CPU sanitizer test runs against a
host-only build) is compiled with gcc, linked with the built library and the
HIP runtime, and run with numeric checks on: every entry point on tiny and
ragged lattices in every storage form and reaction, mass conservation without
reaction, exact forward Euler of uniform fields under a linear reaction,
bitwise round trips of the populations, the tall-lattice launch gate, the
autotuner, batches and the server.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from pathlib import Path

import pytest

pytestmark = pytest.mark.gpu

ROOT = Path(__file__).resolve().parents[1]
PKG = ROOT / "paper_1007_3109_amd"


@pytest.mark.timeout(600)
def test_c_program_through_the_abi(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lib = PKG / "liblbrd.so"
    assert lib.exists(), "liblbrd.so is not built"
    exe = tmp_path / "abi_driver"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", f"-I{ROOT / 'include'}", str(ROOT / "tests" / "abi_driver.c"),
                    "-o", str(exe), f"-L{PKG}", "-llbrd", "-L/opt/rocm/lib", "-lamdhip64", "-lm",
                    f"-Wl,-rpath,{PKG}", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    print("running the C ABI driver on the GPU", flush=True)
    r = subprocess.run([str(exe), "gpu"], capture_output=True, text=True, timeout=540, env=dict(os.environ))
    print(r.stdout[-4000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert "0 failures" in r.stdout
