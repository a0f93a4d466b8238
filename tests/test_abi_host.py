"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates configurations without touching a GPU."""
from __future__ import annotations

import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

from paper_1007_3109_amd import lbrd

HEADER = Path(__file__).resolve().parents[1] / "include" / "lbrd.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbrd_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 30
    lib = ctypes.CDLL(str(lbrd._LIB_PATH))
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(names) == set(lbrd.SIGNATURES), set(names) ^ set(lbrd.SIGNATURES)


def gs(nx=32, ny=32, **kw):
    base = dict(nspecies=2, tau=(1.0, 0.75), storage="f32", reaction="gray_scott", F=0.04, k=0.06)
    base.update(kw)
    return lbrd.make_config(nx, ny, **base)


@pytest.mark.parametrize("mutate", [
    lambda c: setattr(c, "nx", 0),
    lambda c: setattr(c, "ny", -3),
    lambda c: setattr(c, "nspecies", 0),
    lambda c: setattr(c, "nspecies", 5),
    lambda c: setattr(c, "nspecies", 1),            # Gray-Scott needs N = 2
    lambda c: setattr(c, "storage", 7),
    lambda c: setattr(c, "reaction", 9),
    lambda c: setattr(c, "reserved", 1),
    lambda c: c.tau.__setitem__(0, 0.5),            # tau must exceed 1/2
    lambda c: c.tau.__setitem__(1, float("nan")),
    lambda c: setattr(c, "F", float("inf")),
    lambda c: c.u.__setitem__(0, float("nan")),
    lambda c: (c.u.__setitem__(0, 0.5), c.u.__setitem__(1, 0.35)),   # u.u >= 1/3
    lambda c: (setattr(c, "nx", 1 << 16), setattr(c, "ny", (1 << 15) + 1)),   # more than 2^31 sites
])
def test_invalid_configs_rejected(mutate):
    c = gs()
    assert lbrd.validate(c) == lbrd.OK
    mutate(c)
    assert lbrd.validate(c) == lbrd.EINVAL
    n = ctypes.c_size_t()
    assert lbrd.lib.lbrd_workspace_size(ctypes.byref(c), ctypes.byref(n)) == lbrd.EINVAL


def test_advection_velocity_validation():
    """A velocity in the equilibrium is accepted for Gray-Scott and for one
    species (linear or no reaction) with u.u < 1/3; a multi-species linear
    system with a velocity is rejected."""
    assert lbrd.validate(gs(u=(0.1, -0.05))) == lbrd.OK
    assert lbrd.validate(lbrd.make_config(8, 8, 1, tau=0.8, reaction="linear", K=[[-0.01]], u=(0.2, 0.0))) == lbrd.OK
    assert lbrd.validate(lbrd.make_config(8, 8, 1, tau=0.8, u=(0.0, -0.3))) == lbrd.OK
    two = lbrd.make_config(8, 8, 2, tau=0.8, reaction="linear", K=-0.01 * np.eye(2))
    assert lbrd.validate(two) == lbrd.OK
    two.u[0] = 0.1
    assert lbrd.validate(two) == lbrd.EINVAL
    assert lbrd.validate(gs(u=(0.4, 0.42))) == lbrd.EINVAL


def test_shear_flow_validation():
    """A shear flow is accepted for Gray-Scott and one-species linear solvers
    in FP64 / FP32 storage with a whole number of periods and |u| below the
    bound on every row; refused in 16-bit storage, with a fractional or
    missing period count, past the bound, for a multi-species linear system,
    and by batches and the server (single solvers only)."""
    ok = gs(40, 30, u=(0.05, 0.02), shear=(0.2, 3))
    assert lbrd.validate(ok) == lbrd.OK
    assert lbrd.validate(lbrd.make_config(8, 8, 1, tau=0.8, storage="f64", reaction="linear", K=[[-0.01]],
                                          shear=(0.1, 1))) == lbrd.OK
    bad = [gs(40, 30, storage="f16", rho_ref=(1.0, 0.0), shear=(0.1, 1)),
           gs(40, 30, shear=(0.1, 1.5)),
           gs(40, 30, shear=(0.1, 0)),
           gs(40, 30, shear=(0.0, 2)),
           gs(40, 30, u=(0.3, 0.0), shear=(0.3, 1)),
           gs(40, 30, shear=(float("nan"), 1)),
           lbrd.make_config(8, 8, 2, tau=0.8, reaction="linear", K=-0.01 * np.eye(2), shear=(0.1, 1))]
    for c in bad:
        assert lbrd.validate(c) == lbrd.EINVAL
    arr = (lbrd.Config * 1)(ok)
    n = ctypes.c_size_t()
    assert lbrd.lib.lbrd_batch_workspace_size(arr, 1, ctypes.byref(n)) == lbrd.EINVAL
    assert lbrd.lib.lbrd_server_footprint(ctypes.byref(ok), ctypes.byref(n)) == lbrd.EINVAL


def test_workspace_size_covers_two_padded_buffers():
    for storage, b in (("f64", 8), ("f32", 4), ("f16", 2), ("bf16", 2)):
        for nx, ny in ((1, 1), (67, 45), (1024, 1024)):
            c = gs(nx, ny, storage=storage)
            n = lbrd.workspace_size(c)
            assert n >= 2 * 9 * 2 * nx * ny * b
            # padding stays modest for large lattices
            if nx * ny >= 1 << 20:
                assert n <= 1.02 * 2 * 9 * 2 * nx * ny * b + (1 << 20)


def test_linear_and_none_accept_any_species_count():
    for n in range(1, 5):
        assert lbrd.validate(lbrd.make_config(9, 7, n, tau=0.8, reaction="linear", K=-0.01 * __import__("numpy").eye(n))) == 0
        assert lbrd.validate(lbrd.make_config(9, 7, n, tau=0.8, reaction="none")) == 0


def test_batch_and_server_sizes_host_only():
    cfgs = (lbrd.Config * 3)(gs(64, 64), gs(67, 45, storage="f16", rho_ref=(1.0, 0.0)), lbrd.make_config(10, 10, 1, tau=0.9))
    n = ctypes.c_size_t()
    assert lbrd.lib.lbrd_batch_workspace_size(cfgs, 3, ctypes.byref(n)) == 0
    assert n.value >= sum(lbrd.workspace_size(c) for c in cfgs) - 3 * (1 << 16)
    assert lbrd.lib.lbrd_batch_workspace_size(cfgs, 0, ctypes.byref(n)) == lbrd.EINVAL
    assert lbrd.server_footprint(cfgs[0]) >= 2 * 9 * 2 * 64 * 64 * 4 + 2 * 64 * 64 * 8


def test_strerror_names_every_status():
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lbrd.lib.lbrd_strerror(st)
    assert b"gfx950" in lbrd.lib.lbrd_version()


def test_null_handles_are_rejected():
    assert lbrd.lib.lbrd_step(None, 1) == lbrd.EINVAL
    assert lbrd.lib.lbrd_destroy(None) == lbrd.OK
    assert lbrd.lib.lbrd_batch_destroy(None) == lbrd.OK
    assert lbrd.lib.lbrd_server_destroy(None) == lbrd.OK
    c = gs()
    out = ctypes.c_void_p()
    # misaligned or null workspace is refused before any device call
    assert lbrd.lib.lbrd_create(ctypes.byref(c), None, 1 << 30, None, ctypes.byref(out)) == lbrd.EINVAL
    assert lbrd.lib.lbrd_create(ctypes.byref(c), 0x1001, 1 << 30, None, ctypes.byref(out)) == lbrd.EINVAL
    assert lbrd.lib.lbrd_create(ctypes.byref(c), 0x1000, 16, None, ctypes.byref(out)) == lbrd.ENOMEM


def test_binding_shares_torchs_hip_runtime():
    """Importing the binding before torch must not map a second HIP runtime:
    device pointers and streams come from torch, so the library has to bind to
    the runtime torch loads (a second runtime sees neither)."""
    import ast
    import subprocess
    import sys
    code = ("from paper_1007_3109_amd import lbrd\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "print(sorted({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    root = Path(__file__).resolve().parents[1]
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    libs = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs
