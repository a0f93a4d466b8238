"""Gray-Scott parameter map and linear-stability analysis (host-side utilities).

These are the closed forms of Section III of Ayodele, Varnik & Raabe: the
non-dimensionalisation (Eqs. "reac_diff12"-"reac_diff17"), the homogeneous
steady states (Eq. "reac_diff19"), the homogeneous Jacobian and its
eigenvalues (Eqs. "reac_diff24"-"reac_diff26"), and the Turing analysis
(Eqs. "reac_diff29"-"reac_diff34").  No lattice Boltzmann arithmetic lives
here; the workload generators use the classification to draw (F, k) pairs.

Parameter convention (the paper's kinetics with A_0 = k_1 = 1): u = A,
v = B, F = k_f, k = k_2, so R_u = -u v^2 + F (1 - u) and
R_v = u v^2 - (F + k) v.  Then
    tau_A = 1/F, tau_B = 1/(F + k)          (Eq. "reac_diff12")
    B_0 = sqrt(F)                            (Eq. "reac_diff13")
    eta = sqrt(F) / (F + k)                  (after Eq. "reac_diff15")
    tau_GS = tau_A / tau_B = (F + k) / F     (after Eq. "reac_diff17")
    eps^2 = tau_GS * D_u / D_v               (after Eq. "reac_diff17")
and dimensionless fields A~ = u, B~ = v / sqrt(F), time t~ = F t, length
x~ = x / l_A with l_A = sqrt(D_u / F).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class GSDimensionless:
    eta: float
    tau: float      # tau_GS = tau_A / tau_B
    eps2: float     # epsilon_GS^2 = tau_GS * D_u / D_v


def dimensionless(F: float, k: float, Du: float, Dv: float) -> GSDimensionless:
    """(F, k, D_u, D_v) -> (eta, tau_GS, eps_GS^2)."""
    eta = math.sqrt(F) / (F + k)
    tau = (F + k) / F
    return GSDimensionless(eta, tau, tau * Du / Dv)


def feed_kill(eta: float, tau: float) -> tuple[float, float]:
    """Inverse map (eta, tau_GS) -> (F, k): sqrt(F) = 1/(eta tau), k = (tau-1) F."""
    F = 1.0 / (eta * tau) ** 2
    return F, (tau - 1.0) * F


def eta_for_eta_B_minus(x: float) -> float:
    """eta with eta B~- = x (x >= 2): from B~- = (eta + sqrt(eta^2 - 4)) / 2 of
    Eq. "reac_diff19", eta^2 = x^2 / (x - 1)."""
    if x < 2.0:
        raise ValueError("eta B~- >= 2 on the B~- branch")
    return x / math.sqrt(x - 1.0)


def steady_states(eta: float):
    """Homogeneous steady states (A~, B~) of Eq. "reac_diff18".

    Always the trivial (1, 0); for eta >= 2 also (A~+, B~+) and (A~-, B~-) of
    Eq. "reac_diff19": A~± = (eta ± sqrt(eta^2-4)) / (2 eta),
    B~± = (eta ∓ sqrt(eta^2-4)) / 2.  Returns a dict keyed 'trivial', '+', '-'.
    """
    out = {"trivial": (1.0, 0.0)}
    if eta >= 2.0:
        r = math.sqrt(max(eta * eta - 4.0, 0.0))
        out["+"] = ((eta + r) / (2 * eta), (eta - r) / 2)
        out["-"] = ((eta - r) / (2 * eta), (eta + r) / 2)
    return out


def jacobian(eta: float, tau: float, A: float, B: float) -> np.ndarray:
    """Homogeneous Jacobian J of Eq. "reac_diff24" in the paper's printed order
    (first row: the B~ equation scaled by tau; second row: the A~ equation).
    The rows/columns are ordered (B~, A~); trace and determinant do not depend
    on that order."""
    return np.array([[tau * (2 * eta * A * B - 1), tau * eta * B * B],
                     [-2 * A * B, -(B * B + 1)]])


def growth_rates(trace: float, det: float):
    """Eigenvalues alpha_{1,2} = (tr ± sqrt(tr^2 - 4 det)) / 2 (Eq. "reac_diff26")."""
    disc = complex(trace * trace - 4 * det)
    r = disc ** 0.5
    return (trace + r) / 2, (trace - r) / 2


def turing_matrix(eta: float, tau: float, eps2: float, A: float, B: float, q2: float) -> np.ndarray:
    """M(q~) of Eq. "reac_diff29" (same (B~, A~) ordering as ``jacobian``)."""
    return np.array([[tau * (2 * eta * A * B - 1 - q2 / eps2), tau * eta * B * B],
                     [-2 * A * B, -(q2 + B * B + 1)]])


def trace_M(eta: float, tau: float, eps2: float, B: float, q2: float) -> float:
    """tr M(q~^2) = tau - eta B~ - q~^2 (tau/eps^2 + 1) at a non-trivial state."""
    return tau - eta * B - q2 * (tau / eps2 + 1.0)


def det_M(eta: float, tau: float, eps2: float, B: float, q2: float) -> float:
    """|M(q~^2)| = q~^4 tau/eps^2 + q~^2 (tau eta B~/eps^2 - tau) + tau (eta B~ - 2)."""
    return q2 * q2 * tau / eps2 + q2 * (tau * eta * B / eps2 - tau) + tau * (eta * B - 2.0)


def q2_min(eta: float, eps2: float, B: float) -> float:
    """Minimiser of |M(q~^2)|: q~^2_min = (eps^2 - eta B~) / 2 (Eq. "reac_diff31")."""
    return (eps2 - eta * B) / 2.0


def band(eta: float, eps2: float, B: float):
    """Roots q~^2_{1,2} of |M(q~^2)| = 0 (Eq. "reac_diff32"), or None if the
    discriminant is negative (no band)."""
    x = eta * B
    disc = (x - eps2) ** 2 - 4 * eps2 * (x - 2)
    if disc < 0:
        return None
    r = math.sqrt(disc)
    return ((-(x - eps2) - r) / 2.0, (-(x - eps2) + r) / 2.0)


def turing_onset_eps2(x: float) -> float:
    """Smallest eps^2 for which the B~- state has a band of unstable q~^2 > 0,
    with x = eta B~-:  eps^2 > y+(x) = [(6x - 8) + sqrt((6x - 8)^2 - 4 x^2)] / 2.

    Derived from the discriminant of Eq. "reac_diff32" together with
    q~^2_min > 0 (Eq. "reac_diff31").  The paper's printed upper bound of the
    Turing space (Eq. "reac_diff33") is not consistent with that discriminant;
    this exact onset is used instead."""
    d = (6 * x - 8) ** 2 - 4 * x * x
    if d < 0:
        return x   # (6x-8)^2 < 4x^2 only for x < 2, where det M(0) < 0 already
    return max(((6 * x - 8) + math.sqrt(d)) / 2.0, x)


def paper_turing_upper_eps2(x: float) -> float:
    """The paper's printed upper bound -8 + 11.65 x of Eq. "reac_diff33"
    (reported for comparison only; see ``turing_onset_eps2``)."""
    return -8.0 + 11.65 * x


@dataclass(frozen=True)
class Classification:
    eta: float
    tau: float
    eps2: float
    has_nontrivial: bool     # eta >= 2
    hopf_unstable: bool      # tr M(0) > 0 at B~-  <=> tau > eta B~-
    turing_necessary: bool   # eps^2 > eta B~-  (the paper's Turing curve, Eq. "reac_diff34")
    turing_unstable: bool    # exact: a band of q~^2 > 0 with |M| < 0
    eta_B_minus: float


def classify(F: float, k: float, Du: float, Dv: float) -> Classification:
    g = dimensionless(F, k, Du, Dv)
    st = steady_states(g.eta)
    if "-" not in st:
        return Classification(g.eta, g.tau, g.eps2, False, False, False, False, float("nan"))
    _, Bm = st["-"]
    x = g.eta * Bm
    hopf = g.tau > x
    nec = g.eps2 > x
    turing = g.eps2 > turing_onset_eps2(x)
    return Classification(g.eta, g.tau, g.eps2, True, hopf, nec, turing, x)


# ----- lattice-unit forms ---------------------------------------------------

def lattice_state(F: float, k: float, which: str = "-") -> tuple[float, float]:
    """A homogeneous state in lattice fields (u, v) = (A~, sqrt(F) B~)."""
    g = dimensionless(F, k, 1.0, 1.0)
    A, B = steady_states(g.eta)[which]
    return A, math.sqrt(F) * B


def lattice_linearisation(F: float, k: float, Du: float, Dv: float, u: float, v: float, q2: float) -> np.ndarray:
    """Linearised continuum operator in lattice units about (u, v), rows (u, v):
    L(q) = [[-F - v^2 - D_u q^2, -2 u v], [v^2, 2 u v - (F + k) - D_v q^2]]."""
    return np.array([[-F - v * v - Du * q2, -2 * u * v],
                     [v * v, 2 * u * v - (F + k) - Dv * q2]])


def continuum_growth(F: float, k: float, Du: float, Dv: float, u: float, v: float, q2: float) -> float:
    """max Re eig L(q): growth rate per lattice time step of a Fourier mode."""
    return float(np.max(np.linalg.eigvals(lattice_linearisation(F, k, Du, Dv, u, v, q2)).real))


# ----- closed forms used as reference fields ---------------------------------

def point_source_gaussian(L: int, D: float, kappa: float, t: float, x0=None, y0=None) -> np.ndarray:
    """Infinite-domain solution of the decaying point source, Section II.B,
    Eq. "reac_diff5": exp(-r^2 / (4 D t)) / (4 pi D t) * exp(-kappa t), on an
    L x L grid of sites with the source at (x0, y0) (default L // 2)."""
    x0 = L // 2 if x0 is None else x0
    y0 = L // 2 if y0 is None else y0
    x = np.arange(L, dtype=np.float64)[None, :]
    y = np.arange(L, dtype=np.float64)[:, None]
    r2 = (x - x0) ** 2 + (y - y0) ** 2
    return np.exp(-r2 / (4.0 * D * t)) / (4.0 * math.pi * D * t) * math.exp(-kappa * t)
