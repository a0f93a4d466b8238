"""Parameter studies of the paper run as batched GPU jobs.

truncation_error_sweep: the point-source study of Section II.B (Figs. 1c,d
and 2): the relative error E_rho of the lattice solution against the analytic
Gaussian, Eq. "reac_diff5", over a grid of diffusivities D_A and decay rates
kappa, each lattice taken to the same diffusion extent D t = C.  All lattices
run together in one batch (FP64 storage by default); E_rho is reduced on the
device in FP64.
"""
from __future__ import annotations

import time

import numpy as np

from . import analysis, workloads


def truncation_error_sweep(Ds, kappas, C: float = 2.0, L: int = 100, storage: str = "f64", device="cuda"):
    import torch

    from . import lbrd

    Ds = list(Ds)
    kappas = list(kappas)
    cfgs, steps, keys = [], [], []
    for kappa in kappas:
        for D in Ds:
            tau = 3.0 * D + 0.5          # D = c_s^2 (tau - 1/2), c_s^2 = 1/3
            cfgs.append(lbrd.make_config(L, L, 1, tau=tau, storage=storage, reaction="linear", K=[[-kappa]]))
            steps.append(int(round(C / D)))
            keys.append((kappa, D))
    b = lbrd.Batch(cfgs, device=device)
    rho0 = workloads.point_source(L, L, 1)
    for i in range(len(cfgs)):
        b.init(i, rho0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.advance(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    E = np.zeros((len(kappas), len(Ds)))
    for i, (kappa, D) in enumerate(keys):
        ref = torch.tensor(analysis.point_source_gaussian(L, D, kappa, steps[i])[None], device=device)
        E[kappas.index(kappa), Ds.index(D)] = b.rel_l2(i, ref)[0]
    b.close()
    site_steps = L * L * sum(steps)
    return {"E": E, "D": np.array(Ds), "kappa": np.array(kappas), "steps": np.array(steps).reshape(len(kappas), len(Ds)),
            "D_min": np.array(Ds)[np.argmin(E, axis=1)], "seconds": secs, "mlups": site_steps / secs / 1e6}
