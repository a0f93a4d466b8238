"""Batched parameter studies on the GPU against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1007_3109_amd import workloads  # noqa: E402
from pins import gaussian_point_source  # noqa: E402


TRUNCATION_DS = [0.004, 0.006, 0.008, 0.01, 0.012, 0.015, 0.02, 0.025, 0.03, 0.04, 0.05, 0.06]
_D_MIN = {}


@pytest.mark.parametrize("C", [2.0, 4.0, 8.0])
def test_truncation_error_sweep_matches_oracle(C):
    """Section II.B point-source study (Figs. 1c,d) as one FP64 batch, at the
    same diffusive time D t = C for every D (C = 2, 4, 8): every
    E_rho(D, kappa) equals the oracle's within 1e-9 relative (FP64 rounding
    order only), and the minimum over D lies at larger D for the larger
    kappa.  The curves and minima are printed."""
    from paper_1007_3109_amd import studies

    kappas = [0.01, 0.033]
    res = studies.truncation_error_sweep(TRUNCATION_DS, kappas, C=C)
    print(f"C = {C}: {res['E'].size} lattices, {res['seconds']:.3f} s, {res['mlups']:.0f} MLUPS; D_min {res['D_min']}",
          flush=True)
    for a, kappa in enumerate(kappas):
        print(f"  kappa {kappa}: E_rho " + " ".join(f"{d}:{e:.4g}" for d, e in zip(TRUNCATION_DS, res["E"][a])),
              flush=True)
        for j, D in enumerate(TRUNCATION_DS):
            t = int(res["steps"][a, j])
            rho = oracle.solve(workloads.point_source(100, 100, 1), t, [oracle.tau_from_diffusivity(D)],
                               oracle.REACT_LINEAR, K=[-kappa])
            e = oracle.rel_l2(rho, gaussian_point_source(100, D, kappa, t)[None])[0]
            assert abs(res["E"][a, j] - e) <= 1e-9 * e, (C, kappa, D)
    assert res["D_min"][1] > res["D_min"][0]
    _D_MIN[C] = res["D_min"]


def test_truncation_error_minimum_moves_with_the_time_constant():
    """At kappa = 0.01 the error minimum over D moves to larger D as the
    diffusive time C grows (the oracle on the same grid: 0.008, 0.012 and
    0.025 for C = 2, 4, 8); C = 4 puts it at 0.012, the value the paper
    prints for kappa = 0.01."""
    from paper_1007_3109_amd import studies

    mins = {}
    for C in (2.0, 4.0, 8.0):
        mins[C] = _D_MIN.get(C)
        if mins[C] is None:
            mins[C] = studies.truncation_error_sweep(TRUNCATION_DS, [0.01, 0.033], C=C)["D_min"]
    print(f"D_min by C: {mins}", flush=True)
    assert mins[2.0][0] < mins[4.0][0] < mins[8.0][0]
    assert mins[4.0][0] == 0.012


@pytest.mark.parametrize("nx,ny", [(48, 40), (50, 96), (7, 11), (1, 3), (5200, 6)])
def test_spectrum_kernel_matches_numpy_fft(nx, ny):
    """The FP64 power spectrum equals numpy's FFT of the same (read-back)
    density field, mean removed: lines whose length factors into 2, 3 and 5
    take the LDS FFT (48 x 40, 50 x 96, the columns of 5200 x 6), the others
    the direct sums (prime lengths 7 and 11; rows of 5200, longer than the
    LDS holds); a single-site line is its own transform."""
    from paper_1007_3109_amd import lbrd

    rho0 = workloads.gray_scott_square(nx, ny, seed=3)
    cfg = lbrd.make_config(nx, ny, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott", F=0.04, k=0.06)
    s = lbrd.Solver(cfg)
    s.init(rho0).step(300)
    rho = s.moments()[0].cpu().numpy()
    for sp in (0, 1):
        P = s.spectrum(sp).cpu().numpy()
        g = rho[sp] - rho[sp].mean()
        want = np.abs(np.fft.fft2(g)) ** 2
        assert np.abs(P - want).max() <= 1e-9 * max(want.max(), 1e-30), (nx, ny, sp)
    s.close()


def test_phase_diagram_signs_and_band():
    """Section III.D check as a batch: at Hopf-stable points (D_u/D_v = 8)
    the perturbation of (A~-, B~-) decays where the exact Turing analysis says
    stable and grows into a pattern where it says unstable; every grown
    pattern's dominant wavenumber lies in the predicted band (Eq.
    "reac_diff32" mapped to lattice units), within one lattice mode.  One
    instance is checked against the oracle."""
    from paper_1007_3109_amd import analysis, studies

    eta = float(np.sqrt(4.5))           # eta B~- = 3: Turing onset at eps^2 = 9
    points = [(eta, 1.0), (eta, 1.6), (eta, 2.0), (eta, 2.5)]
    res, perf = studies.phase_diagram(points, Du_over_Dv=8.0, L=64, steps=4000)
    print(f"phase diagram: {perf}", flush=True)
    for r in res:
        print({k: v for k, v in r.items() if k != "spectrum"}, flush=True)
        assert not r["hopf_unstable"]
        if r["turing_unstable"]:
            assert r["growth"] > 100
            lo, hi = r["q_band"]
            dq = 2 * np.pi / 64
            assert lo - dq <= r["q"] <= hi + dq
        else:
            assert r["growth"] < 1
    # oracle parity for the tau = 2.0 lattice (FP32 against FP64, with the
    # FP32 rounding floor as in the other Gray-Scott checks)
    from paper_1007_3109_amd import lbrd

    F, k = analysis.feed_kill(eta, 2.0)
    u, v = analysis.lattice_state(F, k, "-")
    rho0 = workloads.perturbed_state(64, 64, u, v, 1e-3, (1, 1))
    taus = [1.0, 3 * (1 / 48) + 0.5]
    s = lbrd.Solver(lbrd.make_config(64, 64, 2, tau=taus, storage="f32", reaction="gray_scott", F=F, k=k))
    s.init(rho0).step(1500)
    got = s.moments()[0].cpu().numpy()
    ref = oracle.solve(rho0, 1500, taus, oracle.REACT_GRAY_SCOTT, F=F, k=k)
    floor = oracle.rel_l2(oracle.solve(rho0, 1500, taus, oracle.REACT_GRAY_SCOTT, precision="f32", F=F, k=k), ref)
    assert np.all(oracle.rel_l2(got, ref) <= np.maximum(1e-5, 3 * floor))


# (eta B~-, tau_GS) at D_u / D_v = 2: the Hopf line is tau_GS = eta B~-
# (tr M(0) = 0), the exact Turing onset eps^2 = 2 tau_GS = y+(eta B~-); each
# point is at least 15 % in tau_GS from both (Turing-only points exist only
# for eta B~- < 16/7)
RATIO2_POINTS = [(2.05, 1.2), (2.05, 1.69), (2.05, 2.6), (2.1, 1.86), (3.0, 2.4), (3.0, 3.75), (3.0, 5.6),
                 (2.2657, 2.733)]


def test_phase_diagram_at_the_papers_ratio():
    """Section III.C-D at the diffusivity ratio of the paper's phase diagram
    (Fig. 6, D_A / D_B = 2), 256^2 lattices from the B~- state with a small
    seed of the zero mode (1e-5 on v) and of the other modes (U(-1e-6, 1e-6),
    no cosine seed): points on both sides of the Hopf line and of the exact
    Turing onset, including the Fig. 7 point.  Hopf-unstable points
    (tr M(0) > 0) grow the zero mode by more than 30x within 1000 steps (its
    linear rate is 0.006 to 0.01 per step) and oscillate: sampled every 30
    steps through the linear stage, it follows the two-term recurrence of the
    forward-Euler map of the linearised reaction, whose fitted roots equal
    that map's complex eigenvalue pair within 5 % (linear periods 209 to 729
    steps; the oracle on 64^2 gives 0.03-2.5 %); Hopf-stable points damp it;
    among the
    Hopf-stable points the Turing-unstable ones grow a pattern (the largest
    non-zero mode by more than 100x in power after 1000 steps, still linear:
    the fastest rates are 0.007 and 0.009 per step, amplitudes stay near
    1e-3, and at the end of the run) whose dominant wavenumber after 1000
    steps lies in the linear band (within one lattice mode), and the others
    decay.  (Saturated, the pattern of the point at tau_GS = 1.69 puts most
    of its power in a mode far below the band by step 6000.)"""
    from paper_1007_3109_amd import analysis, studies

    points = [(analysis.eta_for_eta_B_minus(x), tau) for x, tau in RATIO2_POINTS]
    res, perf = studies.phase_diagram(points, Du_over_Dv=2.0, L=256, steps=6000, phi=0.0, noise=1e-6,
                                      zero_offset=1e-5, probe=1000, samples=200)
    print(f"phase diagram at D_u/D_v = 2: {perf}", flush=True)
    kinds = set()
    for (x, tau), r in zip(RATIO2_POINTS, res):
        zratio = r["zero_probe"] / r["zero_start"]
        print(f"eta B- {x} tau {tau}: hopf {r['hopf_unstable']} turing {r['turing_unstable']} | zero mode x{zratio:.3g} "
              f"after 1000 steps, {r['zero_sign_changes']} sign changes, pattern growth {r['growth_probe']:.3g} "
              f"(mode {r['mode_probe']} q {r['q_probe']:.4f}) after 1000 steps, {r['growth']:.3g} (mode {r['mode']} "
              f"q {r['q']:.4f}) at the end, band {r['q_band']}", flush=True)
        assert abs(r["eta_B_minus"] - x) <= 1e-12 * x
        if r["hopf_unstable"]:
            assert zratio > 30
            # linear stage (samples every 30 steps while the zero mode stays
            # below 1e-4 and the fastest spatial mode below 1e-3, as the
            # linear rates predict): the mean evolves by the forward-Euler map
            # of the linearised reaction, so its samples obey
            # z(k+2) = tr(M) z(k+1) - det(M) z(k) with M = (I + J)^30; the
            # fitted recurrence's roots are M's eigenvalues, a complex pair
            # outside the unit circle (a growing oscillation)
            u_m, v_m = analysis.lattice_state(r["F"], r["k"], "-")
            J = analysis.lattice_linearisation(r["F"], r["k"], 1 / 6, 1 / 12, u_m, v_m, 0.0)
            zrate = float(np.max(np.linalg.eigvals(J).real))
            qs = 2 * np.pi * np.arange(1, 129) / 256
            srate = max(analysis.continuum_growth(r["F"], r["k"], 1 / 6, 1 / 12, u_m, v_m, q * q) for q in qs)
            t_end = min(600.0, np.log(10.0) / zrate, np.log(1e3) / max(srate, 1e-9))
            zs = np.asarray(r["zero_series"][:max(6, int(t_end // 30))])
            (a, b), *_ = np.linalg.lstsq(np.stack([zs[1:-1], zs[:-2]], axis=1), zs[2:], rcond=None)
            fit = np.sort_complex(np.roots([1.0, -a, -b]))
            want = np.sort_complex(np.linalg.eigvals(np.linalg.matrix_power(np.eye(2) + J, 30)))
            print(f"  zero-mode recurrence over {len(zs)} samples: roots {fit}, linear {want}", flush=True)
            assert np.all(np.abs(fit.imag) > 0) and np.all(np.abs(fit) > 1)
            assert np.max(np.abs(fit - want)) <= 0.05 * np.abs(want[0])
        else:
            assert zratio < 1
            if r["turing_unstable"]:
                lo, hi = r["q_band"]
                dq = 2 * np.pi / 256
                assert r["growth_probe"] > 100 and r["growth"] > 100
                assert lo - dq <= r["q_probe"] <= hi + dq
            else:
                assert r["growth"] < 1
        kinds.add((r["hopf_unstable"], r["turing_unstable"]))
    assert kinds == {(False, False), (False, True), (True, False), (True, True)}


def test_rescaling_study_keeps_stripe_count():
    """Section IV (Figs. 11, 12): at the Turing-regime point eta = 2.016933,
    tau_GS = 2.7303 (D_u / D_v = 2), boxes of side 64 .. 256 with both
    diffusivities scaled as (L / 64)^2 and the cos(2 pi x / L) cos(2 pi y / L)
    start keep the stripe count |n| of the dominant mode (q_max L constant
    within 15 %), while a box twice as large with the smaller box's
    diffusivities doubles it.  The smallest lattice equals the FP64 oracle
    within the FP32 rounding floor."""
    from paper_1007_3109_amd import studies

    sizes = [64, 96, 128, 192, 256]
    res = studies.rescaling_study(sizes, 64, (0.03, 0.015), 2.016933, 2.7303, 20000, start="cos")
    ns = {L: res["sizes"][L]["n"] for L in sizes}
    print(f"rescaling: stripe counts {ns}, control {[(k, c['n']) for k, c in res['control_modes'].items()]}, "
          f"{res['seconds']:.2f} s", flush=True)
    med = float(np.median(list(ns.values())))
    assert med > 6                                    # a developed pattern, not the start's mode 1
    for L in sizes:
        assert abs(ns[L] - med) <= 0.15 * med, (L, ns)
    for (L, L2), c in res["control_modes"].items():
        assert abs(c["n"] - 2 * ns[L]) <= 0.25 * 2 * ns[L], (L, L2, c["n"], ns[L])
    # parity of the batched lattice with the oracle (2000 steps, smallest box)
    short = studies.rescaling_study([64, 128], 64, (0.03, 0.015), 2.016933, 2.7303, 2000, start="cos", control=False)
    d = short["sizes"][64]
    taus = [oracle.tau_from_diffusivity(x) for x in d["D"]]
    kw = dict(F=short["F"], k=short["k"])
    ref = oracle.solve(d["init"], 2000, taus, oracle.REACT_GRAY_SCOTT, **kw)
    floor = oracle.rel_l2(oracle.solve(d["init"], 2000, taus, oracle.REACT_GRAY_SCOTT, precision="f32", **kw), ref)
    tol = np.where(floor <= 1e-6, 1e-5, 3 * floor)
    assert np.all(oracle.rel_l2(d["rho"], ref) <= tol), (oracle.rel_l2(d["rho"], ref), floor)


def _line_stripes(row):
    """Stripes crossed along a line: half the sign changes of v - mean(v)."""
    d = np.sign(row - row.mean())
    d[d == 0] = 1
    return int(np.sum(d != np.roll(d, 1))) // 2


def test_stripe_count_over_the_papers_size_range():
    """Section IV, Fig. 12 (text's point eta = 2.014, tau_GS = 2.733, D_u / D_v
    = 2): boxes of side 50 .. 500 with both diffusivities scaled as L^2
    (D_u = 0.0625 at L = 100, so tau_u runs from 0.547 at L = 50 to 5.19 at L =
    500) from the cos start, 400000 steps (the paper's t).  The stripe count
    |n| of the dominant mode stays within 15 % of the linear prediction L
    q_max / 2 pi (12.5, the fastest-growing mode of the linearisation at the
    B~- state) at every size, and the profile of v along y / L = 0.85 spans the
    same range (its maximum within 10 % of the sizes' median, its minimum
    below 0.05).  The profiles themselves do not coincide point by point (the
    labyrinth's orientation and phase differ from size to size): their
    relative gaps are printed, not asserted."""
    from paper_1007_3109_amd import analysis, studies

    sizes = [50, 100, 200, 400, 500]
    eta, tau, Du = 2.014, 2.733, 0.0625
    res = studies.rescaling_study(sizes, 100, (Du, Du / 2), eta, tau, 400000, start="cos", control=False)
    F, k = res["F"], res["k"]
    u, v = analysis.lattice_state(F, k, "-")
    qs = np.linspace(0.01, 1.5, 3000)
    g = [analysis.continuum_growth(F, k, Du, Du / 2, u, v, q * q) for q in qs]
    n_lin = 100 * qs[int(np.argmax(g))] / (2 * np.pi)
    ns = {L: res["sizes"][L]["n"] for L in sizes}
    rows = {L: res["sizes"][L]["v"][int(round(0.85 * L)) % L] for L in sizes}
    tops = {L: float(rows[L].max()) for L in sizes}
    prof = {L: res["sizes"][L]["profile"] for L in sizes}
    gaps = {L: float(np.sqrt(((prof[L] - prof[2 * L]) ** 2).mean() / (prof[2 * L] ** 2).mean()))
            for L in sizes if 2 * L in sizes}
    print(f"sizes {sizes}: |n| {ns} (linear {n_lin:.2f}), stripes along y/L = 0.85 "
          f"{ {L: _line_stripes(rows[L]) for L in sizes} }, v max on the line {tops}, profile gaps L vs 2L {gaps}, "
          f"{res['seconds']:.1f} s", flush=True)
    for L in sizes:
        assert abs(ns[L] - n_lin) <= 0.15 * n_lin, (L, ns, n_lin)
        assert float(rows[L].min()) < 0.05, (L, rows[L].min())
    med = float(np.median(list(tops.values())))
    assert all(abs(t - med) <= 0.1 * med for t in tops.values()), tops
