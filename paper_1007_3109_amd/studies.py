"""Parameter studies of the paper run as batched GPU jobs.

truncation_error_sweep: the point-source study of Section II.B (Figs. 1c,d
and 2): the relative error E_rho of the lattice solution against the analytic
Gaussian, Eq. "reac_diff5", over a grid of diffusivities D_A and decay rates
kappa, each lattice taken to the same diffusion extent D t = C.  All lattices
run together in one batch (FP64 storage by default); E_rho is reduced on the
device in FP64.

phase_diagram: Gray-Scott runs over (eta, tau_GS) points from the perturbed
homogeneous state (Section III.D, Figs. 6-8), with the power spectrum of v
computed on the device and the dominant mode set against the linear-stability
band.

rescaling_study: the length-rescaling test of Section IV (Figs. 10-12): the
same dimensionless (eta, tau_GS, eps) on boxes of side L with every
diffusivity scaled as (L / L_ref)^2 and the start scaled with the box; the
pattern should be the same up to the scale factor (equal stripe or spot
count, q_max L constant, block-averaged fields and normalised profiles
alike), which a control run with unscaled diffusivities does not show.
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
                  noise: float = 1e-4, seed: int = 0, storage: str = "f32", device="cuda", zero_offset: float = 0.0,
                  probe: int = 0, samples: int = 50):
    """Gray-Scott runs over (eta, tau_GS) points as one batch (Section III.D,
    Figs. 6-8): each lattice starts from the homogeneous state (A~-, B~-) plus
    phi cos(2 pi x / L) cos(2 pi y / L), seeded U(-noise, noise) on both
    species and `zero_offset` added to v everywhere (a seed of the zero mode,
    whose growth is the Hopf instability), runs `steps` steps, and reports
    the power spectrum of v, its dominant mode, the growth of the largest
    non-zero mode, the amplitude of the zero mode (|mean v - v-|) at the start,
    after `probe` steps (0: not measured) and at the end, the dominant mode
    and its growth after `probe` steps too (the linear stage, where the
    unstable band of Eq. "reac_diff32" applies; a saturated pattern can put
    its power anywhere), the number of sign changes of mean v - v- at
    `samples` equally spaced times over the run, and the linear stability
    prediction (Hopf line,
    exact Turing onset, band of unstable wavenumbers in lattice units)."""
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
        rho0[1] += zero_offset
        band = analysis.band(c.eta, c.eps2, c.eta_B_minus / c.eta)
        qband = None if band is None else tuple(float(np.sqrt(max(b, 0.0) * F / Du)) for b in band)
        cfgs.append(lbrd.make_config(L, L, 2, tau=taus, storage=storage, reaction="gray_scott", F=F, k=k))
        inits.append(rho0)
        meta.append(dict(eta=eta, tau=tau, F=F, k=k, eta_B_minus=c.eta_B_minus, hopf_unstable=c.hopf_unstable,
                         turing_unstable=c.turing_unstable, q_band=qband, v_minus=v))
    b = lbrd.Batch(cfgs, device=device)
    for i, r in enumerate(inits):
        b.init(i, r)
    sites = float(L * L)

    def zero_mode(i):
        return b.moments(i)[1][1] / sites - meta[i]["v_minus"]

    p0 = [float(b.spectrum(i, 1).max()) for i in range(len(cfgs))]
    z0 = [zero_mode(i) for i in range(len(cfgs))]
    marks = sorted({int(round(steps * (q + 1) / samples)) for q in range(samples)} | ({probe} if probe else set()))
    series = [[] for _ in cfgs]
    zprobe = [None] * len(cfgs)
    mprobe = [(None, None, None)] * len(cfgs)
    done, secs = 0, 0.0
    for mark in marks:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(mark - done)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        done = mark
        for i in range(len(cfgs)):
            z = zero_mode(i)
            series[i].append(z)
            if mark == probe:
                zprobe[i] = abs(z)
                mprobe[i] = dominant_mode(b.spectrum(i, 1).cpu().numpy())
    out = []
    for i, m in enumerate(meta):
        P = b.spectrum(i, 1).cpu().numpy()
        mode, q, pmax = dominant_mode(P)
        zs = np.array(series[i])
        m.update(mode=mode, q=q, growth=pmax / max(p0[i], 1e-300), spectrum=P, zero_start=abs(z0[i]),
                 zero_probe=zprobe[i], zero_end=float(abs(zs[-1])), zero_series=zs, mode_probe=mprobe[i][0],
                 q_probe=mprobe[i][1],
                 growth_probe=None if mprobe[i][2] is None else mprobe[i][2] / max(p0[i], 1e-300),
                 zero_sign_changes=int(np.sum(np.sign(zs[1:]) != np.sign(zs[:-1]))))
        out.append(m)
    b.close()
    return out, {"seconds": secs, "mlups_per_species": 2 * L * L * steps * len(cfgs) / secs / 1e6}


def _block_average(a: np.ndarray, b: int) -> np.ndarray:
    n, L, _ = a.shape
    return a.reshape(n, L // b, b, L // b, b).mean(axis=(2, 4))


def _rel_l2(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    d = (a - b).reshape(a.shape[0], -1)
    r = b.reshape(b.shape[0], -1)
    return np.sqrt((d * d).sum(axis=1) / np.maximum((r * r).sum(axis=1), 1e-300))


def _profile(v: np.ndarray, frac: float, points: int) -> np.ndarray:
    """v along the row y = round(frac L), resampled (periodic linear
    interpolation) at `points` equally spaced positions x / L in [0, 1)."""
    L = v.shape[1]
    row = v[int(round(frac * L)) % v.shape[0]]
    xs = np.arange(points) * L / points
    i0 = np.floor(xs).astype(int)
    w = xs - i0
    return (1 - w) * row[i0 % L] + w * row[(i0 + 1) % L]


def rescaling_study(sizes, L_ref: int, D_ref, eta: float, tau: float, steps: int, start: str = "box",
                    box_ref: int = 20, phi: float = 1e-3, control: bool = True, profile_y: float = 0.85,
                    profile_points: int = 200, storage: str = "f32", device="cuda"):
    """Section IV: Gray-Scott at fixed (eta, tau_GS) (so F and k fixed) on
    boxes of side L in `sizes`, with (D_u, D_v) = (L / L_ref)^2 D_ref.  Start
    "box": the trivial state with a central square of side box_ref L / L_ref at
    u = 0.5, v = 0.25 (Figs. 9, 10); start "cos": the B~- state plus
    phi cos(2 pi x / L) cos(2 pi y / L) on both species (Figs. 7, 11).  All
    lattices run `steps` steps in one batch.  With control=True every size
    that is twice another also runs with the smaller size's diffusivities.

    Returns per size: the initial and final densities (host, FP64), the
    dominant mode (n_x, n_y) of v, its length n (the stripe count), q_max and
    q_max L (Eq. "reac_diff35"), the profile of v along y = profile_y L
    resampled at profile_points positions x / L; for each pair (L, 2L): the
    relative L2 gap between the 2 x 2 block average of the 2L field and the L
    field (rescaled run, and control run), and the control run's mode."""
    import torch

    from . import lbrd

    sizes = sorted(int(L) for L in sizes)
    F, k = analysis.feed_kill(eta, tau)
    runs = []                                  # (L, D, is_control)
    for L in sizes:
        lam = L / L_ref
        runs.append((L, (lam * lam * D_ref[0], lam * lam * D_ref[1]), False))
    if control:
        for L in sizes:
            if 2 * L in sizes:
                lam = L / L_ref
                runs.append((2 * L, (lam * lam * D_ref[0], lam * lam * D_ref[1]), True))
    cfgs, inits = [], []
    for L, D, _ in runs:
        taus = (3 * D[0] + 0.5, 3 * D[1] + 0.5)          # D = (tau - 1/2) / 3
        cfgs.append(lbrd.make_config(L, L, 2, tau=taus, storage=storage, reaction="gray_scott", F=F, k=k))
        if start == "box":
            inits.append(workloads.gs_box(L, int(round(box_ref * L / L_ref))))
        else:
            u, v = analysis.lattice_state(F, k, "-")
            inits.append(workloads.perturbed_state(L, L, u, v, phi, (1, 1)))
    b = lbrd.Batch(cfgs, device=device)
    for i, r in enumerate(inits):
        b.init(i, r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    fields, per_size, control_modes = {}, {}, {}
    for i, (L, D, is_ctrl) in enumerate(runs):
        rho = b.moments(i)[0].cpu().numpy()
        fields[(L, is_ctrl)] = rho
        mode, q, _ = dominant_mode(b.spectrum(i, 1).cpu().numpy())
        if is_ctrl:
            control_modes[(L // 2, L)] = dict(D=D, mode=mode, n=float(np.hypot(*mode)), q_max=q, qL=q * L)
            continue
        per_size[L] = dict(D=D, mode=mode, n=float(np.hypot(*mode)), q_max=q, qL=q * L,
                           profile=_profile(rho[1], profile_y, profile_points), rho=rho, v=rho[1], init=inits[i])
    b.close()
    gaps, control_gaps = {}, {}
    for L in sizes:
        if 2 * L in sizes:
            coarse = fields[(L, False)]
            gaps[(L, 2 * L)] = _rel_l2(_block_average(fields[(2 * L, False)], 2), coarse)
            if control:
                control_gaps[(L, 2 * L)] = _rel_l2(_block_average(fields[(2 * L, True)], 2), coarse)
    site_steps = sum(2 * L * L for L, _, _ in runs) * steps
    return {"F": F, "k": k, "sizes": per_size, "gaps": gaps, "control_gaps": control_gaps,
            "control_modes": control_modes, "seconds": secs, "mlups_per_species": site_steps / secs / 1e6}
