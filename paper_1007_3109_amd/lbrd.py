"""ctypes binding of liblbrd.so (the C ABI of include/lbrd.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (workspaces, density and population
tensors) and the stream; nothing here computes on the CPU.  Importing this
module loads the library and raises ImportError if it has not been built.
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "liblbrd.so"

MAX_SPECIES = 4

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE, ENOTFOUND, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
SPECTRUM_STATIC_MAX_SITES = 1 << 20   # LBRD_SPECTRUM_STATIC_MAX_SITES

STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
REACTION = {"none": 0, "linear": 1, "gray_scott": 2}
DTYPE_F64, DTYPE_F32 = 0, 1


class Config(ctypes.Structure):
    _fields_ = [
        ("nspecies", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("reaction", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("tau", ctypes.c_double * MAX_SPECIES), ("rho_ref", ctypes.c_double * MAX_SPECIES),
        ("K", ctypes.c_double * (MAX_SPECIES * MAX_SPECIES)), ("c", ctypes.c_double * MAX_SPECIES),
        ("F", ctypes.c_double), ("k", ctypes.c_double), ("u", ctypes.c_double * 2),
        ("shear", ctypes.c_double * 2),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("vec", ctypes.c_int32), ("lanes_x", ctypes.c_int32), ("waves", ctypes.c_int32),
        ("nontemporal", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
        ("plain_order", ctypes.c_int32), ("fused_steps", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
        ("tile_cols", ctypes.c_int32), ("tile_strip", ctypes.c_int32), ("march_rows", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k in ("vec", "lanes_x", "waves", "nontemporal", "graph_steps", "blocks_per_cu",
                                              "plain_order", "fused_steps", "tile_rows", "tile_cols", "tile_strip",
                                              "march_rows")}


class ServerConfig(ctypes.Structure):
    _fields_ = [("chunk_steps", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("reserved", ctypes.c_int32), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double), ("steps", ctypes.c_int64),
                ("footprint", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("resident", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("species_site_steps", ctypes.c_int64), ("arena_bytes", ctypes.c_int64),
                ("arena_peak_used", ctypes.c_int64), ("busy_s", ctypes.c_double), ("clock_s", ctypes.c_double),
                ("arena_used", ctypes.c_int64), ("arena_used_byte_s", ctypes.c_double)]


class LbrdError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib.lbrd_strerror(status).decode()} ({status})")


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_PD = ctypes.POINTER(ctypes.c_double)

# every symbol of include/lbrd.h with its argument types
SIGNATURES = {
    "lbrd_strerror": ([_I], ctypes.c_char_p),
    "lbrd_version": ([], ctypes.c_char_p),
    "lbrd_last_error": ([], ctypes.c_char_p),
    "lbrd_validate": ([ctypes.POINTER(Config)], _I),
    "lbrd_workspace_size": ([ctypes.POINTER(Config), ctypes.POINTER(_SZ)], _I),
    "lbrd_create": ([ctypes.POINTER(Config), _P, _SZ, _P, ctypes.POINTER(_P)], _I),
    "lbrd_destroy": ([_P], _I),
    "lbrd_init": ([_P, _P, _I, _I], _I),
    "lbrd_set_populations": ([_P, _P, _I, _I], _I),
    "lbrd_get_populations": ([_P, _P, _I], _I),
    "lbrd_step": ([_P, _I64], _I),
    "lbrd_moments": ([_P, _P, _I, _PD], _I),
    "lbrd_rel_l2": ([_P, _P, _I, _PD], _I),
    "lbrd_time": ([_P, ctypes.POINTER(_I64)], _I),
    "lbrd_spectrum_work_size": ([_I, _I, ctypes.POINTER(_SZ)], _I),
    "lbrd_spectrum": ([_P, _I, _P, _P, _SZ], _I),
    "lbrd_spectrum_static": ([_P, _I, _P], _I),
    "lbrd_get_tuning": ([_P, ctypes.POINTER(Tuning)], _I),
    "lbrd_set_tuning": ([_P, ctypes.POINTER(Tuning)], _I),
    "lbrd_autotune": ([_P, _I, ctypes.c_char_p, ctypes.POINTER(Tuning)], _I),
    "lbrd_time_steps": ([_P, _I64, _PD], _I),
    "lbrd_batch_workspace_size": ([ctypes.POINTER(Config), _I, ctypes.POINTER(_SZ)], _I),
    "lbrd_batch_create": ([ctypes.POINTER(Config), _I, _P, _SZ, _P, ctypes.POINTER(_P)], _I),
    "lbrd_batch_destroy": ([_P], _I),
    "lbrd_batch_init": ([_P, _I, _P, _I, _I], _I),
    "lbrd_batch_moments": ([_P, _I, _P, _I, _PD], _I),
    "lbrd_batch_get_populations": ([_P, _I, _P, _I], _I),
    "lbrd_batch_step": ([_P, _I64], _I),
    "lbrd_batch_advance": ([_P, ctypes.POINTER(_I64)], _I),
    "lbrd_batch_time": ([_P, _I, ctypes.POINTER(_I64)], _I),
    "lbrd_batch_rel_l2": ([_P, _I, _P, _I, _PD], _I),
    "lbrd_batch_spectrum": ([_P, _I, _I, _P, _P, _SZ], _I),
    "lbrd_batch_get_tuning": ([_P, ctypes.POINTER(Tuning)], _I),
    "lbrd_batch_set_tuning": ([_P, ctypes.POINTER(Tuning)], _I),
    "lbrd_batch_autotune": ([_P, _I, ctypes.POINTER(Tuning)], _I),
    "lbrd_batch_time_steps": ([_P, _I64, _PD], _I),
    "lbrd_server_create": ([ctypes.POINTER(ServerConfig), _P, _SZ, _P, ctypes.POINTER(_P)], _I),
    "lbrd_server_destroy": ([_P], _I),
    "lbrd_server_submit": ([_P, ctypes.POINTER(Config), _PD, _I64, ctypes.POINTER(_I64)], _I),
    "lbrd_server_info": ([_P, _I64, ctypes.POINTER(RequestInfo)], _I),
    "lbrd_server_wait": ([_P, _I64, ctypes.c_double], _I),
    "lbrd_server_take": ([_P, _I64, _PD, _PD, ctypes.POINTER(RequestInfo)], _I),
    "lbrd_server_stats_get": ([_P, ctypes.POINTER(ServerStats)], _I),
    "lbrd_server_footprint": ([ctypes.POINTER(Config), ctypes.POINTER(_SZ)], _I),
}


def _load() -> ctypes.CDLL:
    if not _LIB_PATH.exists():
        raise ImportError(f"{_LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    # Device memory and streams come from torch, so the library must bind to the
    # HIP runtime torch carries.  Loading the library first would map the
    # system HIP runtime as well: two runtimes in one process, and the second
    # sees neither torch's allocations nor (once torch holds it) the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(str(_LIB_PATH))
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
lib = _lib


def check(status: int, where: str) -> int:
    if status != OK:
        raise LbrdError(status, where)
    return status


def make_config(nx: int, ny: int, nspecies: int = 1, tau=1.0, storage: str = "f32", reaction: str = "none",
                K=None, c=None, F: float = 0.0, k: float = 0.0, rho_ref=None, u=None, shear=None) -> Config:
    """shear = (A, m): u_x(y) = u[0] + A sin(2 pi m y / ny) on row y."""
    cfg = Config()
    cfg.nspecies, cfg.nx, cfg.ny = nspecies, nx, ny
    cfg.storage = STORAGE[storage]
    cfg.reaction = REACTION[reaction]
    taus = np.broadcast_to(np.asarray(tau, np.float64), (nspecies,))
    for s in range(nspecies):
        cfg.tau[s] = float(taus[s])
    if rho_ref is not None:
        for s, r in enumerate(np.asarray(rho_ref, np.float64).reshape(-1)[:nspecies]):
            cfg.rho_ref[s] = float(r)
    if K is not None:
        Km = np.asarray(K, np.float64).reshape(nspecies, nspecies)
        for s in range(nspecies):
            for j in range(nspecies):
                cfg.K[s * nspecies + j] = float(Km[s, j])
    if c is not None:
        for s, v in enumerate(np.asarray(c, np.float64).reshape(-1)[:nspecies]):
            cfg.c[s] = float(v)
    cfg.F, cfg.k = float(F), float(k)
    if u is not None:
        cfg.u[0], cfg.u[1] = (float(x) for x in u)
    if shear is not None:
        cfg.shear[0], cfg.shear[1] = float(shear[0]), float(shear[1])
    return cfg


def workspace_size(cfg: Config) -> int:
    n = _SZ()
    check(_lib.lbrd_workspace_size(ctypes.byref(cfg), ctypes.byref(n)), "lbrd_workspace_size")
    return n.value


def spectrum_work_size(nx: int, ny: int) -> int:
    n = _SZ()
    check(_lib.lbrd_spectrum_work_size(int(nx), int(ny), ctypes.byref(n)), "lbrd_spectrum_work_size")
    return n.value


def validate(cfg: Config) -> int:
    return _lib.lbrd_validate(ctypes.byref(cfg))


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _device_ptr(t) -> int:
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return int(t.data_ptr())


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return DTYPE_F64
    if t.dtype == torch.float32:
        return DTYPE_F32
    raise ValueError("float64 or float32 expected")


def _alloc_workspace(nbytes: int, device):
    torch = _torch()
    # 256-byte aligned: request a little more and offset
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


class Solver:
    """One periodic lattice.  State lives in a torch-allocated workspace."""

    def __init__(self, cfg: Config, device="cuda", stream=None):
        torch = _torch()
        self.cfg = cfg
        self.device = torch.device(device)
        self.nbytes = workspace_size(cfg)
        self._ws, ptr = _alloc_workspace(self.nbytes, self.device)
        h = _P()
        check(_lib.lbrd_create(ctypes.byref(cfg), ptr, self.nbytes, _stream_handle(stream), ctypes.byref(h)),
              "lbrd_create")
        self._h = h

    @property
    def shape(self):
        return (self.cfg.nspecies, self.cfg.ny, self.cfg.nx)

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbrd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, rho0):
        """rho0: numpy array (host) or device tensor, [N][ny][nx] float64/float32."""
        if isinstance(rho0, np.ndarray):
            a = np.ascontiguousarray(rho0, np.float64)
            assert a.shape == self.shape, (a.shape, self.shape)
            check(_lib.lbrd_init(self._h, a.ctypes.data, DTYPE_F64, 0), "lbrd_init")
        else:
            assert tuple(rho0.shape) == self.shape
            check(_lib.lbrd_init(self._h, _device_ptr(rho0), _dtype_code(rho0), 1), "lbrd_init")
        return self

    def set_populations(self, f):
        if isinstance(f, np.ndarray):
            a = np.ascontiguousarray(f, np.float64)
            assert a.shape == (self.cfg.nspecies, 9, self.cfg.ny, self.cfg.nx)
            check(_lib.lbrd_set_populations(self._h, a.ctypes.data, DTYPE_F64, 0), "lbrd_set_populations")
        else:
            check(_lib.lbrd_set_populations(self._h, _device_ptr(f), _dtype_code(f), 1), "lbrd_set_populations")
        return self

    def get_populations(self, dtype=None):
        torch = _torch()
        out = torch.empty((self.cfg.nspecies, 9, self.cfg.ny, self.cfg.nx), dtype=dtype or torch.float64,
                          device=self.device)
        check(_lib.lbrd_get_populations(self._h, _device_ptr(out), _dtype_code(out)), "lbrd_get_populations")
        return out

    def step(self, n: int = 1):
        check(_lib.lbrd_step(self._h, int(n)), "lbrd_step")
        return self

    def moments(self, dtype=None, mass: bool = True):
        """Returns (rho device tensor [N][ny][nx], FP64 masses as numpy or None)."""
        torch = _torch()
        rho = torch.empty(self.shape, dtype=dtype or torch.float64, device=self.device)
        m = (ctypes.c_double * self.cfg.nspecies)() if mass else None
        st = _lib.lbrd_moments(self._h, _device_ptr(rho), _dtype_code(rho), m)
        if st not in (OK, ENONFINITE):
            check(st, "lbrd_moments")
        return rho, (np.array(m[:]) if mass else None)

    def mass(self) -> np.ndarray:
        m = (ctypes.c_double * self.cfg.nspecies)()
        st = _lib.lbrd_moments(self._h, None, DTYPE_F64, m)
        if st not in (OK, ENONFINITE):
            check(st, "lbrd_moments")
        return np.array(m[:])

    def rel_l2(self, ref) -> np.ndarray:
        e = (ctypes.c_double * self.cfg.nspecies)()
        st = _lib.lbrd_rel_l2(self._h, _device_ptr(ref), _dtype_code(ref), e)
        if st not in (OK, ENONFINITE):
            check(st, "lbrd_rel_l2")
        return np.array(e[:])

    def time(self) -> int:
        t = _I64()
        check(_lib.lbrd_time(self._h, ctypes.byref(t)), "lbrd_time")
        return t.value

    def spectrum(self, species: int):
        """|DFT(rho_s - mean)|^2 as a device float64 tensor [ny][nx]."""
        torch = _torch()
        out = torch.empty((self.cfg.ny, self.cfg.nx), dtype=torch.float64, device=self.device)
        nbytes = spectrum_work_size(self.cfg.nx, self.cfg.ny)
        work, ptr = _alloc_workspace(nbytes, self.device)
        check(_lib.lbrd_spectrum(self._h, int(species), _device_ptr(out), ptr, nbytes), "lbrd_spectrum")
        torch.cuda.current_stream().synchronize()
        del work
        return out

    def spectrum_static(self, species: int, out=None):
        """lbrd_spectrum_static: the same spectrum with the library's fixed
        per-GPU scratch (no allocation in the library; pass `out`, a device
        float64 tensor [ny][nx], to allocate nothing here either).
        Asynchronous on the solver's stream."""
        if out is None:
            torch = _torch()
            out = torch.empty((self.cfg.ny, self.cfg.nx), dtype=torch.float64, device=self.device)
        check(_lib.lbrd_spectrum_static(self._h, int(species), _device_ptr(out)), "lbrd_spectrum_static")
        return out

    def tuning(self) -> Tuning:
        t = Tuning()
        check(_lib.lbrd_get_tuning(self._h, ctypes.byref(t)), "lbrd_get_tuning")
        return t

    def set_tuning(self, **kw):
        t = self.tuning()
        for k, v in kw.items():
            setattr(t, k, v)
        check(_lib.lbrd_set_tuning(self._h, ctypes.byref(t)), "lbrd_set_tuning")
        return self.tuning()

    def autotune(self, steps: int = 20, cache_path: str | None = None) -> Tuning:
        t = Tuning()
        check(_lib.lbrd_autotune(self._h, int(steps), cache_path.encode() if cache_path else None, ctypes.byref(t)),
              "lbrd_autotune")
        return t

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double()
        check(_lib.lbrd_time_steps(self._h, int(n), ctypes.byref(ms)), "lbrd_time_steps")
        return ms.value


class Batch:
    """Many lattices advanced together by persistent launches."""

    def __init__(self, cfgs, device="cuda", stream=None):
        torch = _torch()
        self.cfgs = list(cfgs)
        arr = (Config * len(self.cfgs))(*self.cfgs)
        self._arr = arr
        n = _SZ()
        check(_lib.lbrd_batch_workspace_size(arr, len(self.cfgs), ctypes.byref(n)), "lbrd_batch_workspace_size")
        self.nbytes = n.value
        self.device = torch.device(device)
        self._ws, ptr = _alloc_workspace(self.nbytes, self.device)
        h = _P()
        check(_lib.lbrd_batch_create(arr, len(self.cfgs), ptr, self.nbytes, _stream_handle(stream), ctypes.byref(h)),
              "lbrd_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbrd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, idx: int, rho0):
        if isinstance(rho0, np.ndarray):
            a = np.ascontiguousarray(rho0, np.float64)
            check(_lib.lbrd_batch_init(self._h, idx, a.ctypes.data, DTYPE_F64, 0), "lbrd_batch_init")
        else:
            check(_lib.lbrd_batch_init(self._h, idx, _device_ptr(rho0), _dtype_code(rho0), 1), "lbrd_batch_init")

    def step(self, n: int):
        check(_lib.lbrd_batch_step(self._h, int(n)), "lbrd_batch_step")

    def advance(self, nsteps):
        """Advance instance i by nsteps[i]."""
        arr = (_I64 * len(self.cfgs))(*[int(x) for x in nsteps])
        check(_lib.lbrd_batch_advance(self._h, arr), "lbrd_batch_advance")

    def time(self, idx: int) -> int:
        t = _I64()
        check(_lib.lbrd_batch_time(self._h, idx, ctypes.byref(t)), "lbrd_batch_time")
        return t.value

    def spectrum(self, idx: int, species: int):
        torch = _torch()
        c = self.cfgs[idx]
        out = torch.empty((c.ny, c.nx), dtype=torch.float64, device=self.device)
        nbytes = spectrum_work_size(c.nx, c.ny)
        work, ptr = _alloc_workspace(nbytes, self.device)
        check(_lib.lbrd_batch_spectrum(self._h, idx, int(species), _device_ptr(out), ptr, nbytes),
              "lbrd_batch_spectrum")
        torch.cuda.current_stream().synchronize()
        del work
        return out

    def rel_l2(self, idx: int, ref) -> np.ndarray:
        e = (ctypes.c_double * self.cfgs[idx].nspecies)()
        st = _lib.lbrd_batch_rel_l2(self._h, idx, _device_ptr(ref), _dtype_code(ref), e)
        if st not in (OK, ENONFINITE):
            check(st, "lbrd_batch_rel_l2")
        return np.array(e[:])

    def moments(self, idx: int, dtype=None, mass: bool = True):
        torch = _torch()
        c = self.cfgs[idx]
        rho = torch.empty((c.nspecies, c.ny, c.nx), dtype=dtype or torch.float64, device=self.device)
        m = (ctypes.c_double * c.nspecies)() if mass else None
        st = _lib.lbrd_batch_moments(self._h, idx, _device_ptr(rho), _dtype_code(rho), m)
        if st not in (OK, ENONFINITE):
            check(st, "lbrd_batch_moments")
        return rho, (np.array(m[:]) if mass else None)

    def get_populations(self, idx: int, dtype=None):
        torch = _torch()
        c = self.cfgs[idx]
        out = torch.empty((c.nspecies, 9, c.ny, c.nx), dtype=dtype or torch.float64, device=self.device)
        check(_lib.lbrd_batch_get_populations(self._h, idx, _device_ptr(out), _dtype_code(out)),
              "lbrd_batch_get_populations")
        return out

    def tuning(self) -> Tuning:
        t = Tuning()
        check(_lib.lbrd_batch_get_tuning(self._h, ctypes.byref(t)), "lbrd_batch_get_tuning")
        return t

    def set_tuning(self, **kw):
        t = self.tuning()
        for k, v in kw.items():
            setattr(t, k, v)
        check(_lib.lbrd_batch_set_tuning(self._h, ctypes.byref(t)), "lbrd_batch_set_tuning")
        return self.tuning()

    def autotune(self, steps: int = 10) -> Tuning:
        t = Tuning()
        check(_lib.lbrd_batch_autotune(self._h, int(steps), ctypes.byref(t)), "lbrd_batch_autotune")
        return t

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double()
        check(_lib.lbrd_batch_time_steps(self._h, int(n), ctypes.byref(ms)), "lbrd_batch_time_steps")
        return ms.value


def server_footprint(cfg: Config) -> int:
    n = _SZ()
    check(_lib.lbrd_server_footprint(ctypes.byref(cfg), ctypes.byref(n)), "lbrd_server_footprint")
    return n.value


class Server:
    """Continuous-batching solve server over a torch-allocated device arena."""

    def __init__(self, arena_bytes: int, chunk_steps: int = 500, max_slots: int = 4096, max_queue: int = 1 << 20,
                 device="cuda", stream=None):
        torch = _torch()
        self.device = torch.device(device)
        self._arena, ptr = _alloc_workspace(int(arena_bytes), self.device)
        sc = ServerConfig(int(chunk_steps), int(max_slots), int(max_queue), 0)
        h = _P()
        check(_lib.lbrd_server_create(ctypes.byref(sc), ptr, int(arena_bytes), _stream_handle(stream),
                                      ctypes.byref(h)), "lbrd_server_create")
        self._h = h
        self._shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            check(_lib.lbrd_server_destroy(self._h), "lbrd_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, cfg: Config, rho0: np.ndarray, nsteps: int) -> int:
        a = np.ascontiguousarray(rho0, np.float64)
        assert a.shape == (cfg.nspecies, cfg.ny, cfg.nx)
        t = _I64()
        check(_lib.lbrd_server_submit(self._h, ctypes.byref(cfg), a.ctypes.data_as(_PD), int(nsteps),
                                      ctypes.byref(t)), "lbrd_server_submit")
        self._shapes[t.value] = (cfg.nspecies, cfg.ny, cfg.nx)
        return t.value

    def info(self, ticket: int) -> RequestInfo:
        i = RequestInfo()
        check(_lib.lbrd_server_info(self._h, int(ticket), ctypes.byref(i)), "lbrd_server_info")
        return i

    def wait(self, ticket: int, timeout_s: float = 600.0):
        check(_lib.lbrd_server_wait(self._h, int(ticket), float(timeout_s)), "lbrd_server_wait")

    def take(self, ticket: int):
        shape = self._shapes.pop(ticket)
        rho = np.empty(shape, np.float64)
        m = np.empty(shape[0], np.float64)
        i = RequestInfo()
        st = _lib.lbrd_server_take(self._h, int(ticket), rho.ctypes.data_as(_PD), m.ctypes.data_as(_PD),
                                   ctypes.byref(i))
        if st not in (OK, ENONFINITE):
            check(st, "lbrd_server_take")
        return rho, m, i

    def stats(self) -> ServerStats:
        s = ServerStats()
        check(_lib.lbrd_server_stats_get(self._h, ctypes.byref(s)), "lbrd_server_stats_get")
        return s
