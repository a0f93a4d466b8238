"""Oracle for the reacting-species D2Q9 lattice Boltzmann update.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never imports, links or calls it, and this package imports nothing
from the product.

The arithmetic lives in ``lbrd_oracle.c`` (plain loops, FP64, push form of the
update equation of Section II.A, second Eq. "relax"; Appendix Eq. "app1").  This
module only marshals numpy arrays through ctypes and adds the read-outs that
the paper defines on top of the populations:

* ``moments``: rho_s = sum_i f_{i,s} (Section II.A, after Eq. "relax");
* ``mass``: M_s = sum_x rho_s(x), an exactly rounded FP64 sum (math.fsum);
* ``rel_l2``: the relative error E_rho of Section II.B (the equation after
  Eq. "reac_diff5"), computed per species.

Functions without a pin in the test-suite say so in their docstring; every
function here is pinned (see tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_BUILD = _HERE / "_build"
_LIB = _BUILD / "liboracle.so"

REACT_NONE = 0
REACT_LINEAR = 1
REACT_GRAY_SCOTT = 2

Q_NONE = 0
Q_F16 = 1
Q_BF16 = 2

MAX_SPECIES = 4


def build(force: bool = True) -> Path:
    """Compile the oracle (FP64 and FP32 builds of the same source) with gcc.

    No fast-math and no FMA contraction: the FP64 build is plain IEEE double
    with round-to-nearest-even in source order.
    """
    _BUILD.mkdir(exist_ok=True)
    if _LIB.exists() and not force:
        return _LIB
    src = _HERE / "lbrd_oracle.c"
    objs = []
    flags = ["-O2", "-fPIC", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11"]
    for real, sfx in (("double", "f64"), ("float", "f32")):
        obj = _BUILD / f"oracle_{sfx}.o"
        subprocess.run(
            ["gcc", *flags, f"-DREAL={real}", f"-DSFX(name)=name##_{sfx}", "-c", str(src), "-o", str(obj)],
            check=True,
        )
        objs.append(str(obj))
    tmp = _BUILD / "liboracle.so.tmp"
    subprocess.run(["gcc", "-shared", "-fopenmp", *objs, "-o", str(tmp), "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build()
        lib = ctypes.CDLL(str(_LIB))
        for sfx, ct in (("f64", ctypes.c_double), ("f32", ctypes.c_float)):
            P = ctypes.POINTER(ct)
            pd = ctypes.POINTER(ctypes.c_double)
            pi = ctypes.POINTER(ctypes.c_int)
            getattr(lib, f"orc_tables_{sfx}").argtypes = [P, pi, pi]
            getattr(lib, f"orc_init_{sfx}").argtypes = [ctypes.c_int] * 3 + [pd, pd, ctypes.c_int, P]
            fn = getattr(lib, f"orc_run_{sfx}")
            fn.argtypes = ([ctypes.c_int] * 3 + [pd, ctypes.c_int, pd, ctypes.c_int, pd, pd, ctypes.c_int, P, P,
                                                  ctypes.c_int64])
            getattr(lib, f"orc_eq_coefs_{sfx}").argtypes = [pd, P]
            fn.restype = ctypes.c_int
            getattr(lib, f"orc_moments_{sfx}").argtypes = [ctypes.c_int] * 3 + [P, pd]
            getattr(lib, f"orc_threads_{sfx}").restype = ctypes.c_int
            getattr(lib, f"orc_encode_{sfx}").argtypes = [ctypes.c_int] * 4 + [pd, pd, P]
            pf = ctypes.POINTER(ctypes.c_float)
            getattr(lib, f"orc_quantise_{sfx}").argtypes = [ctypes.c_int, pf, pf, ctypes.c_int64]
        _lib = lib
    return _lib


def _dt(precision: str):
    if precision == "f64":
        return np.float64, ctypes.c_double
    if precision == "f32":
        return np.float32, ctypes.c_float
    raise ValueError(precision)


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def threads() -> int:
    """OpenMP threads the oracle's step runs on."""
    return int(_load().orc_threads_f64())


def tables(precision: str = "f64"):
    """The oracle's D2Q9 tables: (w[9], ex[9], ey[9]) (Eq. "Weights")."""
    npdt, ct = _dt(precision)
    w = np.zeros(9, npdt)
    ex = np.zeros(9, np.int32)
    ey = np.zeros(9, np.int32)
    getattr(_load(), f"orc_tables_{precision}")(_ptr(w, ct), _ptr(ex, ctypes.c_int), _ptr(ey, ctypes.c_int))
    return w, ex, ey


def _velocity(u):
    """None, the 2 components of a uniform equilibrium velocity, or a
    prescribed field [ny][nx][2], as a C array."""
    if u is None:
        return None
    a = np.asarray(u, np.float64)
    return np.ascontiguousarray(a if a.ndim == 3 else a.reshape(2))


def _is_field(ua) -> int:
    return int(ua is not None and ua.ndim == 3)


def _uptr(a):
    return None if a is None else _ptr(a, ctypes.c_double)


def eq_coefs(u=None, precision: str = "f64") -> np.ndarray:
    """The oracle's equilibrium coefficients c_i(u) of Eq. "Maxwellian"
    (f^eq_i = c_i rho; c_i = w_i when u is None or zero)."""
    npdt, ct = _dt(precision)
    c = np.zeros(9, npdt)
    ua = _velocity(u)
    getattr(_load(), f"orc_eq_coefs_{precision}")(_uptr(ua), _ptr(c, ct))
    return c


def init(rho0: np.ndarray, precision: str = "f64", u=None) -> np.ndarray:
    """Equilibrium populations f_{i,s} = c_i(u) rho0_s (c_i = w_i without a
    velocity; u uniform or a field [ny][nx][2]), shape [N][9][ny][nx]."""
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    n, ny, nx = rho0.shape
    npdt, ct = _dt(precision)
    f = np.zeros((n, 9, ny, nx), npdt)
    ua = _velocity(u)
    if _is_field(ua):
        assert ua.shape == (ny, nx, 2)
    getattr(_load(), f"orc_init_{precision}")(n, nx, ny, _ptr(rho0, ctypes.c_double), _uptr(ua), _is_field(ua),
                                              _ptr(f, ct))
    return f


def _params(reaction: int, n: int, K=None, c=None, F=None, k=None) -> np.ndarray:
    if reaction == REACT_LINEAR:
        Km = np.zeros((n, n)) if K is None else np.asarray(K, np.float64).reshape(n, n)
        cv = np.zeros(n) if c is None else np.asarray(c, np.float64).reshape(n)
        return np.ascontiguousarray(np.concatenate([Km.ravel(), cv]))
    if reaction == REACT_GRAY_SCOTT:
        return np.array([F, k], np.float64)
    return np.zeros(1, np.float64)


def run(f: np.ndarray, nsteps: int, tau, reaction: int = REACT_NONE, *, K=None, c=None, F=None, k=None,
        quant: int = Q_NONE, rho_ref=None, u=None) -> np.ndarray:
    """Advance populations f [N][9][ny][nx] by nsteps; returns a new array.

    The dtype of f selects the build (float64: the oracle proper; float32: the
    rounding-floor / storage-emulation build).  ``quant`` (float32 only) rounds
    every stored population to binary16 or bfloat16 after subtracting
    c_i * rho_ref[s], the 16-bit shifted storage form.  ``u`` is the
    equilibrium velocity of Eq. "Maxwellian" (None: the paper's u = 0; two
    values: uniform; an array [ny][nx][2]: a prescribed field).
    """
    f = np.array(f, copy=True, order="C")
    precision = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}[f.dtype]
    _, ct = _dt(precision)
    n, q, ny, nx = f.shape
    assert q == 9
    tau = np.ascontiguousarray(np.broadcast_to(np.asarray(tau, np.float64), (n,)))
    params = _params(reaction, n, K, c, F, k)
    rref = np.zeros(n) if rho_ref is None else np.ascontiguousarray(np.asarray(rho_ref, np.float64).reshape(n))
    if quant != Q_NONE and precision != "f32":
        raise ValueError("storage emulation runs in the float build")
    work = np.empty_like(f)
    ua = _velocity(u)
    if _is_field(ua):
        assert ua.shape == (ny, nx, 2)
        if quant != Q_NONE:
            raise ValueError("the storage emulation takes a uniform velocity")
    rc = getattr(_load(), f"orc_run_{precision}")(
        n, nx, ny, _ptr(tau, ctypes.c_double), reaction, _ptr(params, ctypes.c_double), quant,
        _ptr(rref, ctypes.c_double), _uptr(ua), _is_field(ua), _ptr(f, ct), _ptr(work, ct), int(nsteps))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return f


def encode(f: np.ndarray, quant: int, rho_ref, u=None) -> np.ndarray:
    """Populations in the 16-bit shifted storage form (float build):
    c_i rho_ref_s + Q(f - c_i rho_ref_s); returns a new float32 array."""
    f = np.array(f, dtype=np.float32, copy=True, order="C")
    n, _, ny, nx = f.shape
    rref = np.ascontiguousarray(np.asarray(rho_ref, np.float64).reshape(n))
    ua = _velocity(u)
    _load().orc_encode_f32(n, nx, ny, quant, _ptr(rref, ctypes.c_double), _uptr(ua), _ptr(f, ctypes.c_float))
    return f


def quantise(x: np.ndarray, quant: int) -> np.ndarray:
    """Round float32 values to binary16 (Q_F16) or bfloat16 (Q_BF16), ties to
    even, returned as float32 (the oracle's storage emulation)."""
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty_like(x)
    _load().orc_quantise_f32(quant, _ptr(x, ctypes.c_float), _ptr(out, ctypes.c_float), x.size)
    return out


def moments(f: np.ndarray) -> np.ndarray:
    """rho_s(x) = sum_{i=0..8} f_{i,s}(x), summed in ascending i; float64 [N][ny][nx]."""
    f = np.ascontiguousarray(f)
    precision = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}[f.dtype]
    _, ct = _dt(precision)
    n, _, ny, nx = f.shape
    rho = np.zeros((n, ny, nx), np.float64)
    getattr(_load(), f"orc_moments_{precision}")(n, nx, ny, _ptr(f, ct), _ptr(rho, ctypes.c_double))
    return rho


def mass(rho: np.ndarray) -> np.ndarray:
    """Total mass per species, M_s = sum_x rho_s(x), correctly rounded (fsum)."""
    return np.array([math.fsum(np.asarray(r, np.float64).ravel().tolist()) for r in rho])


def rel_l2(rho: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-species relative L2 error E = sqrt(sum |ref - rho|^2 / sum |ref|^2)
    (Section II.B, the definition of E_rho), accumulated in FP64."""
    rho = np.asarray(rho, np.float64)
    ref = np.asarray(ref, np.float64)
    out = []
    for a, b in zip(rho, ref):
        num = math.fsum(((b - a) ** 2).ravel().tolist())
        den = math.fsum((b ** 2).ravel().tolist())
        out.append(math.sqrt(num / den) if den > 0 else math.sqrt(num))
    return np.array(out)


def tau_from_diffusivity(D: float) -> float:
    """tau_s from D_s = c_s^2 (tau_s - 1/2) with c_s^2 = 1/3, dt = 1 (Section II.A,
    the last sentence of the subsection; Appendix Eq. "app23")."""
    return 3.0 * D + 0.5


def solve(rho0: np.ndarray, nsteps: int, tau, reaction: int = REACT_NONE, precision: str = "f64", **kw):
    """Convenience: equilibrium init, nsteps of the update, density read-out."""
    f = init(rho0, precision, kw.get("u"))
    f = run(f, nsteps, tau, reaction, **kw)
    return moments(f)
