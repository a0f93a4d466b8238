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


def dominant_mode(P: np.ndarray):
    """(n_x, n_y) of the largest non-zero Fourier component of a power
    spectrum P[k_y][k_x], with n in (-L/2, L/2], and its wavenumber
    q = 2 pi sqrt((n_x/L_x)^2 + (n_y/L_y)^2) (Section III.D, Eq. "reac_diff35")."""
    P = np.array(P, dtype=np.float64, copy=True)
    P[0, 0] = 0.0
    ky, kx = np.unravel_index(int(np.argmax(P)), P.shape)
    ny, nx = P.shape
    n_x = kx if kx <= nx // 2 else kx - nx
    n_y = ky if ky <= ny // 2 else ky - ny
    return (n_x, n_y), 2 * np.pi * np.hypot(n_x / nx, n_y / ny), float(P[ky, kx])


def phase_diagram(points, Du_over_Dv: float = 8.0, L: int = 64, steps: int = 4000, phi: float = 1e-3,
                  noise: float = 1e-4, seed: int = 0, storage: str = "f32", device="cuda"):
    """Gray-Scott runs over (eta, tau_GS) points as one batch (Section III.D,
    Figs. 6-8): each lattice starts from the homogeneous state (A~-, B~-) plus
    phi cos(2 pi x / L) cos(2 pi y / L) and seeded U(-noise, noise) on both
    species, runs `steps` steps, and reports the power spectrum of v, its
    dominant mode, the growth of the largest non-zero mode, and the linear
    stability prediction (Hopf line, exact Turing onset, band of unstable
    wavenumbers in lattice units)."""
    import torch

    from . import lbrd

    Du = 1.0 / 6.0                     # tau_u = 1
    Dv = Du / Du_over_Dv
    taus = (3 * Du + 0.5, 3 * Dv + 0.5)
    rng = np.random.default_rng(seed)
    cfgs, inits, meta = [], [], []
    for eta, tau in points:
        F, k = analysis.feed_kill(eta, tau)
        c = analysis.classify(F, k, Du, Dv)
        u, v = analysis.lattice_state(F, k, "-")
        rho0 = workloads.perturbed_state(L, L, u, v, phi, (1, 1)) + rng.uniform(-noise, noise, size=(2, L, L))
        band = analysis.band(c.eta, c.eps2, c.eta_B_minus / c.eta)
        qband = None if band is None else tuple(float(np.sqrt(max(b, 0.0) * F / Du)) for b in band)
        cfgs.append(lbrd.make_config(L, L, 2, tau=taus, storage=storage, reaction="gray_scott", F=F, k=k))
        inits.append(rho0)
        meta.append(dict(eta=eta, tau=tau, F=F, k=k, hopf_unstable=c.hopf_unstable, turing_unstable=c.turing_unstable,
                         q_band=qband))
    b = lbrd.Batch(cfgs, device=device)
    for i, r in enumerate(inits):
        b.init(i, r)
    p0 = [float(b.spectrum(i, 1).max()) for i in range(len(cfgs))]
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    out = []
    for i, m in enumerate(meta):
        P = b.spectrum(i, 1).cpu().numpy()
        mode, q, pmax = dominant_mode(P)
        m.update(mode=mode, q=q, growth=pmax / max(p0[i], 1e-300), spectrum=P)
        out.append(m)
    b.close()
    return out, {"seconds": secs, "mlups_per_species": 2 * L * L * steps * len(cfgs) / secs / 1e6}
