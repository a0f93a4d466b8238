"""Pins of the oracle's float build and of its 16-bit storage emulation."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1007_3109_amd import workloads


def _bf16_neighbours(x: np.ndarray):
    """The two bfloat16 values bracketing each float32 (truncation and the next
    value up in magnitude), from the bit pattern."""
    b = x.view(np.uint32) & np.uint32(0xFFFF0000)
    lo = b.view(np.float32)
    hi = (b + np.uint32(0x10000)).view(np.float32)
    return lo, hi


def test_f16_rounding_matches_numpy():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.normal(0, 1, 20000).astype(np.float32),
        rng.normal(0, 1e-5, 5000).astype(np.float32),      # subnormal range of binary16
        (rng.integers(-2048, 2048, 4000) * np.float32(2.0 ** -12) + np.float32(2.0 ** -13)).astype(np.float32),  # ties
        np.array([0.0, -0.0, 65504.0, 65519.0, 65520.0, 1e-8, -6.1e-5], np.float32),
    ])
    got = oracle.quantise(x, oracle.Q_F16)
    want = x.astype(np.float16).astype(np.float32)   # numpy casts round to nearest even
    assert np.array_equal(got, want)


def test_bf16_rounding_is_nearest_even():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 5000)]).astype(np.float32)
    got = oracle.quantise(x, oracle.Q_BF16)
    lo, hi = _bf16_neighbours(np.abs(x))
    a = np.abs(x).astype(np.float64)
    dlo, dhi = a - lo, hi.astype(np.float64) - a
    even_lo = ((lo.view(np.uint32) >> 16) & 1) == 0
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(even_lo, lo, hi)))
    want = np.copysign(pick, x).astype(np.float32)
    assert np.array_equal(got, want)


def test_float_build_tracks_f64_on_linear_decay():
    rho0 = workloads.sinusoid(64, 64, 0.1, 1)
    r64 = oracle.solve(rho0, 1000, 1.0, oracle.REACT_LINEAR, K=[-1e-3])
    r32 = oracle.solve(rho0, 1000, 1.0, oracle.REACT_LINEAR, precision="f32", K=[-1e-3])
    e = oracle.rel_l2(r32, r64)[0]
    assert 1e-9 < e < 1e-5


def test_storage_emulation_error_scales_with_format():
    """Shifted 16-bit storage: the error against FP64 is larger for bfloat16
    (8 significand bits) than for binary16 (11 bits), and both stay bounded."""
    rho0 = workloads.gray_scott_square(64, 64, seed=3)
    kw = dict(F=0.04, k=0.06)
    r64 = oracle.solve(rho0, 200, [1.0, 0.75], oracle.REACT_GRAY_SCOTT, **kw)
    errs = {}
    for q in (oracle.Q_F16, oracle.Q_BF16):
        f = oracle.encode(oracle.init(rho0, "f32"), q, [1.0, 0.0])
        r = oracle.moments(oracle.run(f, 200, [1.0, 0.75], oracle.REACT_GRAY_SCOTT, quant=q, rho_ref=[1.0, 0.0], **kw))
        errs[q] = oracle.rel_l2(r, r64)
    assert np.all(errs[oracle.Q_F16] < errs[oracle.Q_BF16])
    assert np.all(errs[oracle.Q_F16] < 1e-2)


def test_encode_is_the_storage_rounding():
    """encode() leaves w_i rho_ref + Q(f - w_i rho_ref): the stored 16-bit value
    recovered from it is exactly quantise(f - shift)."""
    rng = np.random.default_rng(4)
    f = rng.uniform(0, 0.5, size=(2, 9, 3, 5)).astype(np.float32)
    w, _, _ = oracle.tables("f32")
    rref = np.array([1.0, 0.25])
    for q in (oracle.Q_F16, oracle.Q_BF16):
        g = oracle.encode(f, q, rref)
        shift = (w[None, :, None, None] * rref.astype(np.float32)[:, None, None, None]).astype(np.float32)
        want = shift + oracle.quantise(f - shift, q)
        assert np.array_equal(g, want.astype(np.float32))
