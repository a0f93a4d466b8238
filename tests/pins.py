"""Independent references used to pin the oracle (test helpers only).

Nothing here calls the oracle's arithmetic.  The Fourier propagator is the
update equation of Section II.A (second Eq. "relax") transformed to Fourier
space by hand: for the discrete transform g^(q) = sum_x g(x) e^{-i q.x}, the
streaming f(x + e_i, t+1) = g(x) becomes f^(q, t+1) = e^{-i q.e_i} g^(q), and a
linear reaction R = J rho + c acts on each mode separately (c only on q = 0).
"""
from __future__ import annotations

import math
import re
from fractions import Fraction
from pathlib import Path

import numpy as np

GOLDEN = Path(__file__).resolve().parent / "golden"


def golden(name: str = "paper_values.txt") -> dict:
    """Parse key = value lines (values: numbers, fractions or space-separated lists)."""
    out = {}
    for line in (GOLDEN / name).read_text().splitlines():
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, val = (s.strip() for s in line.split("=", 1))
        parts = val.split()
        vals = [float(Fraction(p)) for p in parts]
        out[key] = vals[0] if len(vals) == 1 else vals
    return out


def maxwellian_coefs(u, w, ex, ey) -> np.ndarray:
    """c_i(u) = w_i [1 + 3 e_i.u + 9/2 (e_i.u)^2 - 3/2 u.u]: Eq. "Maxwellian"
    with c_s^2 = 1/3, written out with the constants folded (independent of the
    oracle's own expression)."""
    ux, uy = u
    eu = np.asarray(ex, float) * ux + np.asarray(ey, float) * uy
    return np.asarray(w, float) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))


def propagator(q, taus, J, w, ex, ey, ceq=None) -> np.ndarray:
    """One-step Fourier propagator P(q) of the update for a linear reaction
    R_s = sum_r J[s][r] rho_r (9N x 9N, species-major, velocity index i); the
    equilibrium is ceq_i rho (ceq = w without a velocity)."""
    qx, qy = q
    n = len(taus)
    ceq = w if ceq is None else ceq
    P = np.zeros((9 * n, 9 * n), complex)
    for s in range(n):
        om = 1.0 / taus[s]
        for i in range(9):
            row = 9 * s + i
            ph = np.exp(-1j * (qx * ex[i] + qy * ey[i]))
            P[row, row] += ph * (1.0 - om)
            for j in range(9):
                P[row, 9 * s + j] += ph * ceq[i] * om
            for r in range(n):
                for j in range(9):
                    P[row, 9 * r + j] += ph * w[i] * J[s][r]
    return P


def row_field_propagator(qx, ny, tau, kappa, w, ex, ey, ceq_rows) -> np.ndarray:
    """One-step propagator of one species with the decay R = -kappa rho for a
    Fourier mode exp(i qx x) when the equilibrium coefficients depend on the
    row only (ceq_rows[y][i]): the state is the complex amplitude A[i][y]
    (index i * ny + y).  Collision on row y: (1 - 1/tau) A_i + (c_i(y) / tau -
    kappa w_i) sum_j A_j; then the post-collision amplitude moves to row
    y + e_iy and picks up exp(-i qx e_ix)."""
    om = 1.0 / tau
    M = np.zeros((9 * ny, 9 * ny), complex)
    for i in range(9):
        ph = np.exp(-1j * qx * ex[i])
        for y in range(ny):
            yd = (y + ey[i]) % ny
            row = i * ny + yd
            M[row, i * ny + y] += ph * (1.0 - om)
            for j in range(9):
                M[row, j * ny + y] += ph * (ceq_rows[y][i] * om - kappa * w[i])
    return M


def source_vector(c, w, ex, ey, npts) -> np.ndarray:
    """Affine part at q = 0: the constant source c_s enters every site, so its
    q = 0 transform is npts * c_s, weighted by w_i (the phase is 1 at q = 0)."""
    n = len(c)
    v = np.zeros(9 * n, complex)
    for s in range(n):
        for i in range(9):
            v[9 * s + i] = w[i] * c[s] * npts
    return v


def gs_reaction(rho, F, k):
    """Gray-Scott kinetics with A_0 = k_1 = 1 (Section III, Eqs. "reac_diff10",
    "reac_diff11" with k_f = F, k_2 = k)."""
    u, v = rho
    return np.stack([-u * v * v + F * (1 - u), u * v * v - (F + k) * v])


def gs_jacobian(u, v, F, k):
    return np.array([[-v * v - F, -2 * u * v], [v * v, 2 * u * v - (F + k)]])


def gaussian_point_source(L, D, kappa, t, x0=None, y0=None):
    """Infinite-domain solution of Section II.B, Eq. "reac_diff5"."""
    x0 = L // 2 if x0 is None else x0
    y0 = L // 2 if y0 is None else y0
    x = np.arange(L)[None, :]
    y = np.arange(L)[:, None]
    r2 = (x - x0) ** 2 + (y - y0) ** 2
    return np.exp(-r2 / (4 * D * t)) / (4 * math.pi * D * t) * math.exp(-kappa * t)
