"""Seeded synthetic inputs: initial density fields and parameter sets.

This module holds no lattice Boltzmann arithmetic.  It is the only code that
the oracle side (tests, baselines) and the device side share: both receive the
same float64 arrays from these generators.

Every random draw uses ``numpy.random.default_rng`` with a recorded seed.
The workloads follow the paper's synthetic set-ups:

* a sinusoidal mode on a uniform background under a linear decay reaction
  (the analytic-decay check of the linear reaction, Section II.B);
* a point source (Section II.B: a unit density at the centre of a 100 x 100
  periodic box, zero elsewhere);
* the Gray-Scott square perturbation of the trivial state (Section IV: a
  central square with u = 0.5, v = 0.25 in a domain at u = 1, v = 0), plus
  i.i.d. additive U(-0.01, 0.01) noise on both species.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import analysis

# Gray-Scott defaults of the 1024^2 / 4096^2 workloads: D_u / D_v = 2 through
# tau_u = 1.0 (D_u = 1/6) and tau_v = 0.75 (D_v = 1/12).
GS_TAU = (1.0, 0.75)
GS_F = 0.04
GS_K = 0.06


def sinusoid(nx: int, ny: int, amplitude: float = 0.1, mode: int = 1, background: float = 1.0) -> np.ndarray:
    """rho0[0][y][x] = background + amplitude * sin(2 pi mode x / nx); shape [1][ny][nx]."""
    x = np.arange(nx, dtype=np.float64)
    row = background + amplitude * np.sin(2.0 * math.pi * mode * x / nx)
    return np.ascontiguousarray(np.broadcast_to(row, (1, ny, nx)))


def shear_field(nx: int, ny: int, u=(0.0, 0.0), amp: float = 0.0, m: int = 1) -> np.ndarray:
    """Prescribed velocity field [ny][nx][2] of a sinusoidal shear flow:
    u_x = u[0] + amp sin(2 pi m y / ny), u_y = u[1] (the field the solver's
    ``shear`` option describes, for the oracle side)."""
    phase = (m * np.arange(ny)) % ny   # whole periods: the phase in integers
    field = np.empty((ny, nx, 2), np.float64)
    field[..., 0] = (u[0] + amp * np.sin(2.0 * np.pi * phase / ny))[:, None]
    field[..., 1] = u[1]
    return field


def point_source(nx: int, ny: int, nspecies: int = 2) -> np.ndarray:
    """Species 0 is 1 at (nx//2, ny//2) and 0 elsewhere; other species are 0."""
    rho = np.zeros((nspecies, ny, nx))
    rho[0, ny // 2, nx // 2] = 1.0
    return rho


def square_bounds(side: int) -> tuple[int, int]:
    """Central perturbation square [lo, hi) along each axis: a 64-site square
    for sides >= 128, and [side/4, 3 side/4) below that."""
    if side >= 128:
        return side // 2 - 32, side // 2 + 32
    return side // 4, (3 * side) // 4


def gray_scott_square(nx: int, ny: int | None = None, seed: int = 0, noise: float = 0.01,
                      rng: np.random.Generator | None = None) -> np.ndarray:
    """Gray-Scott initial state [2][ny][nx]: u = 1, v = 0 with a central square
    at u = 0.5, v = 0.25, plus additive U(-noise, noise) on both species."""
    ny = nx if ny is None else ny
    rho = np.zeros((2, ny, nx))
    rho[0] = 1.0
    xlo, xhi = square_bounds(nx)
    ylo, yhi = square_bounds(ny)
    rho[0, ylo:yhi, xlo:xhi] = 0.5
    rho[1, ylo:yhi, xlo:xhi] = 0.25
    if noise:
        g = np.random.default_rng(seed) if rng is None else rng
        rho += g.uniform(-noise, noise, size=rho.shape)
    return rho


def gs_box(side: int, box: int, u_in: float = 0.5, v_in: float = 0.25) -> np.ndarray:
    """Noiseless Gray-Scott start [2][side][side]: u = 1, v = 0 with a central
    box x box square at (u_in, v_in) (the finite perturbation of the trivial
    state of Section IV, Fig. 9), rows and columns [side/2 - box/2, +box)."""
    rho = np.zeros((2, side, side))
    rho[0] = 1.0
    lo = side // 2 - box // 2
    rho[0, lo:lo + box, lo:lo + box] = u_in
    rho[1, lo:lo + box, lo:lo + box] = v_in
    return rho


def perturbed_state(nx: int, ny: int, u: float, v: float, amp: float, mode=(1, 1)) -> np.ndarray:
    """Homogeneous (u, v) plus amp * cos(2 pi mx x/nx) cos(2 pi my y/ny) on both
    species (the small-amplitude start of Section III.D)."""
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    p = amp * np.cos(2 * math.pi * mode[0] * x / nx) * np.cos(2 * math.pi * mode[1] * y / ny)
    return np.stack([u + p, v + p])


# ----- batched sweep ----------------------------------------------------------

BATCH_SIDES = (128, 192, 256, 384, 512)


@dataclass
class Instance:
    idx: int
    side: int
    F: float
    k: float
    tau: tuple = GS_TAU
    storage: str = "f32"
    reaction: str = "gray_scott"
    nsteps: int = 0
    K: tuple = field(default_factory=tuple)
    seed: object = None


def batch_sweep(seed: int = 0, grid: int = 16, sides=BATCH_SIDES) -> list[Instance]:
    """The 16 x 16 (F, k) sweep: instance 16 i + j has F_i = 0.01 + 0.07 i/15 and
    k_j = 0.04 + 0.03 j/15; each side is drawn in instance order from
    default_rng(seed) among ``sides``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(grid):
        for j in range(grid):
            F = 0.01 + 0.07 * i / (grid - 1)
            k = 0.04 + 0.03 * j / (grid - 1)
            side = int(rng.choice(np.asarray(sides)))
            out.append(Instance(idx=grid * i + j, side=side, F=F, k=k, seed=[seed, grid * i + j]))
    return out


def batch_initial(inst: Instance) -> np.ndarray:
    """Initial state of one sweep instance, from its own stream default_rng([seed, idx])."""
    return gray_scott_square(inst.side, inst.side, rng=np.random.default_rng(inst.seed))


# ----- serving request stream -------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    side: int
    nsteps: int
    reaction: str           # "linear" or "gray_scott"
    storage: str            # "f32" or "f16"
    tau: tuple
    K: float = 0.0          # decay rate for "linear"
    F: float = 0.0
    k: float = 0.0
    seed: object = None


def draw_gs_unstable(rng: np.random.Generator, Du_over_Dv: float = 2.0, max_tries: int = 10000):
    """(F, k) from the sweep box [0.01, 0.08] x [0.04, 0.07], rejection-sampled
    until the B~- state exists and is Hopf- or Turing-unstable."""
    for _ in range(max_tries):
        F = rng.uniform(0.01, 0.08)
        k = rng.uniform(0.04, 0.07)
        c = analysis.classify(F, k, Du_over_Dv, 1.0)
        if c.has_nontrivial and c.eta > 2.0 and (c.hopf_unstable or c.turing_unstable):
            return F, k
    raise RuntimeError("no unstable (F, k) found")


def request_stream(n: int, rate: float, seed: int = 0, side_range=(64, 2048), steps_range=(1000, 50000)) -> list[Request]:
    """Poisson arrivals (exponential gaps of mean 1/rate).  Half the requests are
    single-species linear decay (kappa ~ U[1e-4, 1e-2], tau ~ U[0.55, 1.5],
    sinusoid of mode 1), half Gray-Scott with (F, k) from ``draw_gs_unstable``;
    side = round(exp(U[ln lo, ln hi])); steps ~ U{lo..hi}; storage f32 or f16
    with probability 1/2 each."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate)
        side = int(round(math.exp(rng.uniform(math.log(side_range[0]), math.log(side_range[1])))))
        nsteps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        storage = "f32" if rng.random() < 0.5 else "f16"
        if rng.random() < 0.5:
            kappa = rng.uniform(1e-4, 1e-2)
            tau = rng.uniform(0.55, 1.5)
            out.append(Request(rid, t, side, nsteps, "linear", storage, (tau,), K=kappa, seed=[seed, rid]))
        else:
            F, k = draw_gs_unstable(rng)
            out.append(Request(rid, t, side, nsteps, "gray_scott", storage, GS_TAU, F=F, k=k, seed=[seed, rid]))
    return out


def request_initial(req: Request) -> np.ndarray:
    if req.reaction == "linear":
        return sinusoid(req.side, req.side, amplitude=0.1, mode=1)
    return gray_scott_square(req.side, req.side, rng=np.random.default_rng(req.seed))
