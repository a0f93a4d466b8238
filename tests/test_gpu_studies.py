"""Batched parameter studies on the GPU against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1007_3109_amd import workloads  # noqa: E402
from pins import gaussian_point_source  # noqa: E402


def test_truncation_error_sweep_matches_oracle():
    """Section II.B point-source study as one FP64 batch: every E_rho(D, kappa)
    equals the oracle's within 1e-9 relative (FP64 rounding order only), and
    the minimum over D moves to larger D when kappa grows."""
    from paper_1007_3109_amd import studies

    Ds = [0.004, 0.006, 0.008, 0.01, 0.012, 0.015, 0.02, 0.025, 0.03, 0.04]
    kappas = [0.01, 0.033]
    res = studies.truncation_error_sweep(Ds, kappas, C=2.0)
    print(f"sweep: {res['E'].size} lattices, {res['seconds']:.3f} s, {res['mlups']:.0f} MLUPS; D_min {res['D_min']}",
          flush=True)
    for a, kappa in enumerate(kappas):
        for j, D in enumerate(Ds):
            t = int(res["steps"][a, j])
            rho = oracle.solve(workloads.point_source(100, 100, 1), t, [oracle.tau_from_diffusivity(D)],
                               oracle.REACT_LINEAR, K=[-kappa])
            e = oracle.rel_l2(rho, gaussian_point_source(100, D, kappa, t)[None])[0]
            assert abs(res["E"][a, j] - e) <= 1e-9 * e, (kappa, D)
    assert res["D_min"][1] > res["D_min"][0]
