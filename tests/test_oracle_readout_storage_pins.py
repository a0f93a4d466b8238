"""Pins of the oracle's read-outs and of its 16-bit storage emulation.

Every GPU parity threshold passes through ``oracle.rel_l2`` and, for the 16-bit
storage forms, through the oracle's emulation of that storage.  These tests fix
both against values worked out by hand or by an independent brute force:

* ``rel_l2`` is E_rho of Section II.B (the equation after Eq. "reac_diff5"):
  sqrt(sum (rho_ref - rho)^2 / sum rho_ref^2), per species.  Hand values with
  exact binary fractions catch a dropped square root, swapped arguments, a
  norm over all species at once or a wrong branch for an empty reference.
* ``mass`` is M_s = sum_x rho_s(x); exact cases with cancellation.
* The storage emulation is one time step of the update (Section II.A, second
  Eq. "relax") in float arithmetic, the result stored as the deviation
  g - w_i rho_ref rounded to binary16 or bfloat16.  A brute force below does
  the same step with numpy float32 arrays, numpy's own binary16 cast and a
  bfloat16 rounding that picks the nearer of the two bracketing values: the
  oracle's float build must equal it bit for bit.
* Fixed point: a uniform field at rho = rho_ref without reaction is an
  equilibrium of the update, so every stored deviation stays exactly zero.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle

F32 = np.float32


# ----- E_rho (Section II.B) ---------------------------------------------------

def test_rel_l2_hand_values():
    ref = np.array([[[3.0, 4.0]]])                      # |ref| = 5
    assert oracle.rel_l2(np.zeros_like(ref), ref)[0] == 1.0
    assert oracle.rel_l2(np.array([[[3.0, 0.0]]]), ref)[0] == 0.8     # sqrt(16/25); no root gives 0.64
    assert oracle.rel_l2(np.array([[[0.0, 4.0]]]), ref)[0] == 0.6
    # the denominator is the reference's norm, not the tested field's
    assert oracle.rel_l2(np.array([[[6.0, 8.0]]]), ref)[0] == 1.0     # swapped arguments give 0.5
    assert oracle.rel_l2(ref, np.array([[[6.0, 8.0]]]))[0] == 0.5


def test_rel_l2_relative_perturbation_is_exact():
    """rho = ref (1 + eps) with binary fractions: E = |eps| exactly."""
    rng = np.random.default_rng(0)
    ref = 2.0 ** rng.integers(-6, 6, size=(3, 17, 23)).astype(np.float64)
    ref *= np.where(rng.random(ref.shape) < 0.5, -1.0, 1.0)
    eps = np.array([2.0 ** -10, -2.0 ** -3, 2.0 ** -20])
    rho = ref * (1.0 + eps[:, None, None])
    got = oracle.rel_l2(rho, ref)
    assert np.array_equal(got, np.abs(eps))               # per species, in order


def test_rel_l2_per_species_and_uniform_offset():
    """Two species with different errors; an offset c on a field of ones gives
    E = c (sum c^2 / sum 1 = c^2)."""
    ref = np.ones((2, 10, 10))
    rho = ref + np.array([0.5, 0.125])[:, None, None]
    assert np.array_equal(oracle.rel_l2(rho, ref), np.array([0.5, 0.125]))
    # a norm over both species at once would give sqrt((25 + 1.5625)/200) for both
    rho[1] = ref[1]
    assert np.array_equal(oracle.rel_l2(rho, ref), np.array([0.5, 0.0]))


def test_rel_l2_empty_reference_is_absolute_norm():
    """A species whose reference is zero everywhere has no relative error; the
    oracle then reports the absolute L2 norm of the difference."""
    ref = np.zeros((2, 1, 2))
    ref[0] = [[3.0, 4.0]]
    rho = np.array([[[3.0, 4.0]], [[3.0, 4.0]]])
    assert np.array_equal(oracle.rel_l2(rho, ref), np.array([0.0, 5.0]))


def test_mass_is_exact_with_cancellation():
    rho = np.array([[[1e16, 1.0, -1e16, 0.5]], [[0.1, 0.2, 0.3, -0.6]]])
    m = oracle.mass(rho)
    assert m[0] == 1.5                                    # a running float sum gives 0.5
    exact = sum(Fraction(x) for x in (0.1, 0.2, 0.3, -0.6))   # the binary values' exact sum
    assert m[1] == float(exact) and m[1] != 0.1 + 0.2 + 0.3 - 0.6
    assert oracle.mass(np.full((1, 8, 8), 0.25))[0] == 16.0


# ----- the 16-bit storage emulation: brute force -----------------------------

def _f16(x):
    """binary16 nearest-even, via numpy's cast."""
    return x.astype(np.float16).astype(F32)


def _bf16(x):
    """bfloat16 nearest-even: the nearer of the two bfloat16 values around x
    (the truncated bit pattern and the next one up in magnitude), the one with
    an even last bit on a tie."""
    a = np.abs(x).astype(F32)
    lo_bits = a.view(np.uint32) & np.uint32(0xFFFF0000)
    lo = lo_bits.view(F32)
    hi = (lo_bits + np.uint32(0x10000)).view(F32)
    dlo = a.astype(np.float64) - lo.astype(np.float64)
    dhi = hi.astype(np.float64) - a.astype(np.float64)
    even_lo = ((lo_bits >> np.uint32(16)) & np.uint32(1)) == 0
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(even_lo, lo, hi)))
    return np.copysign(pick, x).astype(F32)


ROUND = {oracle.Q_F16: _f16, oracle.Q_BF16: _bf16}
W32 = np.array([F32(4) / F32(9)] + [F32(1) / F32(9)] * 4 + [F32(1) / F32(36)] * 4, F32)
EXY = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def _brute_step(f, tau, reaction, params, rref, rnd):
    """One step of the update in float32, stored in the shifted 16-bit form.
    f: float32 [N][9][ny][nx] already in storage form; rnd None: no storage
    rounding (the plain float step)."""
    n = f.shape[0]
    rho = []
    for s in range(n):
        acc = np.zeros(f.shape[2:], F32)
        for i in range(9):
            acc = acc + f[s, i]
        rho.append(acc)
    if reaction == oracle.REACT_GRAY_SCOTT:
        F, k = F32(params[0]), F32(params[1])
        uvv = rho[0] * rho[1] * rho[1]
        R = [-uvv + F * (F32(1) - rho[0]), uvv - (F + k) * rho[1]]
    else:
        K, c = params
        R = []
        for s in range(n):
            acc = np.zeros(f.shape[2:], F32)
            for j in range(n):
                acc = acc + F32(K[s][j]) * rho[j]
            R.append(acc + F32(c[s]))
    out = np.empty_like(f)
    for s in range(n):
        for i, (ex, ey) in enumerate(EXY):
            fi = f[s, i]
            g = fi + (W32[i] * rho[s] - fi) / F32(tau[s]) + W32[i] * R[s]
            if rnd is not None:
                shift = W32[i] * F32(rref[s])
                g = shift + rnd(g - shift)
            out[s, i] = np.roll(g, shift=(ey, ex), axis=(0, 1))     # push to x + e_i, periodic
    return out


def _brute_encode(f, rref, rnd):
    out = np.empty_like(f)
    for s in range(f.shape[0]):
        for i in range(9):
            shift = W32[i] * F32(rref[s])
            out[s, i] = shift + rnd(f[s, i] - shift)
    return out


CASES = [
    ((1, 3), oracle.REACT_GRAY_SCOTT, (0.04, 0.06), [1.0, 0.0], [0.7, 1.2]),
    ((3, 3), oracle.REACT_GRAY_SCOTT, (0.03, 0.055), [1.0, 0.25], [1.0, 0.75]),
    ((2, 5), oracle.REACT_LINEAR, ([[-0.01, 0.002], [0.01, -0.003]], [0.001, -0.0005]), [0.5, 0.0], [0.55, 1.6]),
    ((1, 1), oracle.REACT_LINEAR, ([[-0.02]], [0.0]), [1.0], [0.9]),
]


@pytest.mark.parametrize("quant", [oracle.Q_F16, oracle.Q_BF16])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_storage_emulation_equals_brute_force(quant, case):
    (ny, nx), reaction, params, rref, tau = CASES[case]
    n = len(rref)
    rnd = ROUND[quant]
    rng = np.random.default_rng(100 + case)
    w64 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f = (w64[None, :, None, None] * np.asarray(rref)[:, None, None, None]
         + rng.uniform(-0.02, 0.06, size=(n, 9, ny, nx))).astype(F32)
    f = _brute_encode(f, rref, rnd)
    if reaction == oracle.REACT_GRAY_SCOTT:
        kw = dict(F=params[0], k=params[1])
    else:
        kw = dict(K=params[0], c=params[1])
    # the oracle's encode() is the same storage rounding
    assert np.array_equal(oracle.encode(f, quant, rref), f)
    got = f
    want = f
    for step in range(4):
        got = oracle.run(got, 1, tau, reaction, quant=quant, rho_ref=rref, **kw)
        want = _brute_step(want, tau, reaction, params, rref, rnd)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (step, np.abs(got - want).max())
    # several steps in one call are the same as single steps
    assert np.array_equal(oracle.run(f, 4, tau, reaction, quant=quant, rho_ref=rref, **kw), got)


def test_brute_force_step_is_the_plain_float_step_without_rounding():
    """The brute force without the 16-bit rounding is the oracle's float build
    itself: the storage rounding is the only difference it models."""
    (ny, nx), reaction, params, rref, tau = CASES[1]
    rng = np.random.default_rng(7)
    f = rng.uniform(0.0, 0.3, size=(2, 9, ny, nx)).astype(F32)
    want = _brute_step(f, tau, reaction, params, rref, None)
    got = oracle.run(f, 1, tau, reaction, F=params[0], k=params[1])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("quant", [oracle.Q_F16, oracle.Q_BF16])
@pytest.mark.parametrize("rref,tau", [([1.0, 0.25], [1.0, 0.75]), ([0.5, 2.0], [0.6, 1.7])])
def test_shifted_storage_uniform_reference_is_a_fixed_point(quant, rref, tau):
    """A uniform field at rho_s = rho_ref,s without reaction is an equilibrium of
    the update; in the shifted form all its deviations are zero and must stay
    exactly zero (rounding f itself instead of f - w_i rho_ref would move
    w_i rho_ref = 4/9, 1/9, 1/36 to the nearest 16-bit values)."""
    rho0 = np.asarray(rref)[:, None, None] * np.ones((2, 6, 7))
    f0 = oracle.encode(oracle.init(rho0, "f32"), quant, rref)
    shift = (W32[None, :, None, None] * np.asarray(rref, F32)[:, None, None, None]).astype(F32)
    assert np.array_equal(f0, np.broadcast_to(shift, f0.shape))
    f = oracle.run(f0, 100, tau, oracle.REACT_NONE, quant=quant, rho_ref=rref)
    assert np.array_equal(f, f0)
    f = oracle.run(f0, 100, tau, oracle.REACT_LINEAR, K=np.zeros((2, 2)), quant=quant, rho_ref=rref)
    assert np.array_equal(f, f0)
