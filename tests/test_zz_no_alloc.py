"""lbrd_spectrum_static, the spectrum entry point that allocates nothing (its
scratch is a fixed array the library holds in each GPU's memory), against
lbrd_spectrum (scratch from a caller's work buffer) on the same solver state,
through the C ABI.  Two calls in a row on two solvers, the second lattice
smaller than the first (the array keeps the first call's contents): the power
spectra must be bitwise equal, since both run the same kernels on the same
inputs with a fixed reduction order.  A lattice beyond the array's limit is
refused with ENOMEM before any GPU work."""
from __future__ import annotations

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1007_3109_amd import workloads  # noqa: E402

if torch.cuda.is_available():
    from paper_1007_3109_amd import lbrd  # noqa: E402


def _compare(nx, ny, steps, seed):
    rho0 = workloads.gray_scott_square(nx, ny, seed=seed)
    cfg = lbrd.make_config(nx, ny, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott",
                           F=workloads.GS_F, k=workloads.GS_K)
    s = lbrd.Solver(cfg)
    s.init(rho0).step(steps)
    for species in (1, 0):
        want = s.spectrum(species)
        out = torch.full((ny, nx), float("nan"), dtype=torch.float64, device="cuda")
        rc = lbrd.lib.lbrd_spectrum_static(s._h, species, out.data_ptr())
        assert rc == lbrd.OK, lbrd.lib.lbrd_strerror(rc)
        torch.cuda.synchronize()
        print(f"{nx}x{ny} species {species}: static-scratch spectrum, max {float(out.max()):.6e}", flush=True)
        assert torch.equal(out, want)
    s.close()


def test_static_scratch_spectrum_equals_workspace_spectrum():
    _compare(96, 80, 120, seed=1)
    _compare(40, 36, 30, seed=2)


def test_static_scratch_spectrum_refuses_lattices_beyond_its_array():
    assert 1025 * 1024 > lbrd.SPECTRUM_STATIC_MAX_SITES
    cfg = lbrd.make_config(1025, 1024, 1, tau=0.8, storage="f16", reaction="none", rho_ref=(1.0,))
    s = lbrd.Solver(cfg)
    out = torch.empty((1024, 1025), dtype=torch.float64, device="cuda")
    assert lbrd.lib.lbrd_spectrum_static(s._h, 0, out.data_ptr()) == lbrd.ENOMEM
    s.close()
