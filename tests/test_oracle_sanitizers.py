"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its C
source and a driver that calls every entry point on tiny and ragged lattices
(every reaction kind, both 16-bit storage emulations, with and without an
equilibrium velocity) are built with gcc -fsanitize=address,undefined and run
on the CPU; any out-of-bounds access, leak or undefined operation fails."""
from __future__ import annotations

import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers(tmp_path):
    src = ROOT / "oracle" / "lbrd_oracle.c"
    driver = ROOT / "tests" / "oracle_sanitize_driver.c"
    flags = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
             "-ffp-contract=off", "-std=c11"]
    objs = []
    for real, sfx in (("double", "f64"), ("float", "f32")):
        obj = tmp_path / f"oracle_{sfx}.o"
        subprocess.run(["gcc", *flags, f"-DREAL={real}", f"-DSFX(name)=name##_{sfx}", "-c", str(src), "-o", str(obj)],
                       check=True)
        objs.append(str(obj))
    exe = tmp_path / "driver"
    subprocess.run(["gcc", *flags, str(driver), *objs, "-o", str(exe), "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
