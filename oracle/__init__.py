"""FP64 CPU oracle of the SAC/SMAUG+ MHD scheme -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library neither imports nor
links it, and the two share no code: the oracle is a plain C program
(``sacx_oracle.c``) built with gcc -O2 -ffp-contract=off, driven from here
through ctypes.  Inputs come from the neutral ``workloads`` package.

Parity status: every function is pinned by the CPU test-suite against closed
forms, invariants and brute force, except the hyper-diffusion constants and
the Brio-Wu solution beyond self-consistency ("parity unpinned": no values
exist outside this oracle).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sacx_oracle.c")
# SACX_ORACLE_LIB points the tests at another build of the same source (the
# mutation test builds copies with planted mistakes and runs the pins on them)
_LIB = os.environ.get("SACX_ORACLE_LIB") or os.path.join(_HERE, "libsacx_oracle.so")

FIELDS = ("rho", "mx", "my", "e", "bx", "by")
BACKGROUND_FIELDS = ("rho_b", "e_b", "bx_b", "by_b")

OK = 0
EINVAL = -1
ENONPHYS = -4
ENOMEM = -7

PERIODIC = 0
OPEN = 1

# Arithmetic forms of the scheme (see sacx_oracle.c).  PAPER defines the
# oracle: classic RK4 combined as printed from four kept right-hand sides,
# every division written as a division.  LOWSTORE is the algebraically equal
# four-array arrangement with reciprocals of the grid constants, rho and
# gamma - 1; a device implementation that follows that operation sequence can
# be compared with it bit for bit.  The CPU pins tie the two together.
PAPER = 0
LOWSTORE = 1

# Hyper-diffusion constants (our choice; the paper gives none).  Order of the
# classes: density, thermal energy, velocity, magnetic field.
DEFAULT_C2 = (0.02, 0.02, 0.2, 0.02)
DEFAULT_CSHK = (0.5, 0.5, 0.5, 0.5)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP, no FMA contraction),
    the 3-D oracle beside it."""
    from . import oracle3d
    oracle3d.build(force=force)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("hd_on", ctypes.c_int), ("hd_cross_on", ctypes.c_int),
        ("c2", ctypes.c_double * 4), ("cshk", ctypes.c_double * 4),
        ("bc", ctypes.c_int * 4),
        ("background_on", ctypes.c_int),
        ("g", ctypes.c_double * 2),
        ("form", ctypes.c_int),
    ]


_lib = None
_lock = threading.Lock()
_P = ctypes.POINTER(ctypes.c_double)
_PP = ctypes.POINTER(_P)


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            lib = ctypes.CDLL(_LIB)
            lib.orc_advance.argtypes = [ctypes.POINTER(_Cfg), _PP, _PP, ctypes.c_int, ctypes.c_double,
                                        _P, ctypes.POINTER(ctypes.c_int), _P]
            lib.orc_wavespeed.argtypes = [ctypes.POINTER(_Cfg), _PP, _PP, _P]
            lib.orc_rhs.argtypes = [ctypes.POINTER(_Cfg), _PP, _PP, ctypes.c_double, _PP]
            lib.orc_step_patch.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, ctypes.c_int, _PP, _PP,
                                           ctypes.c_double, ctypes.c_double, _PP]
            lib.orc_sums.argtypes = [ctypes.POINTER(_Cfg), _PP, _P]
            lib.orc_deriv_line.argtypes = [ctypes.c_int, _P, ctypes.c_double, _P]
            lib.orc_hd_ratio_line.argtypes = [ctypes.c_int, _P, _P]
            _F = ctypes.POINTER(ctypes.c_float)
            _I = ctypes.POINTER(ctypes.c_int)
            lib.orc_advance_ext.argtypes = [ctypes.POINTER(_Cfg), _PP, ctypes.c_int, ctypes.c_double,
                                            _P, _I, _P, _F]
            lib.orc_rhs_ext.argtypes = [ctypes.POINTER(_Cfg), _PP, ctypes.c_double, _PP, _F]
            lib.orc_hd_ratio_fields.argtypes = [ctypes.POINTER(_Cfg), _PP, _PP, _P]
            lib.orc_hd_face_fields.argtypes = [ctypes.POINTER(_Cfg), _PP, _PP, _P, _P]
            lib.orc_hd_check.argtypes = [ctypes.POINTER(_Cfg), _PP, _F, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, _I, _I, _P, _P]
            for name in ("orc_advance", "orc_wavespeed", "orc_rhs", "orc_step_patch", "orc_sums",
                         "orc_deriv_line", "orc_hd_ratio_line", "orc_abi_version", "orc_advance_ext",
                         "orc_rhs_ext", "orc_hd_ratio_fields", "orc_hd_check", "orc_hd_face_fields"):
                getattr(lib, name).restype = ctypes.c_int
            _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


def _ptrs(arrs: Sequence[np.ndarray]):
    arr_t = _P * len(arrs)
    return arr_t(*[a.ctypes.data_as(_P) for a in arrs])


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def make_cfg(prob, cfl: float = 0.3, hd_on: bool = True, hd_cross_on: bool = True,
             c2: Sequence[float] = DEFAULT_C2, cshk: Sequence[float] = DEFAULT_CSHK,
             gamma: Optional[float] = None, form: int = PAPER) -> _Cfg:
    c = _Cfg()
    c.nx, c.ny = prob.nx, prob.ny
    c.x0, c.x1, c.y0, c.y1 = prob.x0, prob.x1, prob.y0, prob.y1
    c.gamma = prob.gamma if gamma is None else gamma
    c.cfl = cfl
    c.hd_on = int(bool(hd_on))
    c.hd_cross_on = int(bool(hd_cross_on))
    c.c2 = (ctypes.c_double * 4)(*c2)
    c.cshk = (ctypes.c_double * 4)(*cshk)
    c.bc = (ctypes.c_int * 4)(*prob.bc)
    c.background_on = int(prob.background is not None)
    c.g = (ctypes.c_double * 2)(*getattr(prob, "g", (0.0, 0.0)))
    if form not in (PAPER, LOWSTORE):
        raise ValueError(f"unknown arithmetic form {form!r}")
    c.form = form
    return c


class State:
    """An oracle run: the problem, the scheme constants and the current state."""

    def __init__(self, prob, cfl: float = 0.3, hd_on: bool = True, hd_cross_on: bool = True,
                 c2: Sequence[float] = DEFAULT_C2, cshk: Sequence[float] = DEFAULT_CSHK,
                 form: int = PAPER):
        self.prob = prob
        self.cfg = make_cfg(prob, cfl, hd_on, hd_cross_on, c2, cshk, form=form)
        self.f = [_c64(prob.fields[k]).copy() for k in FIELDS]
        self.bg = None
        if prob.background is not None:
            self.bg = [_c64(prob.background[k]).copy() for k in BACKGROUND_FIELDS]
        self.t = float(prob.t0)
        self.steps = 0
        self.last = np.zeros(4)

    def _bgp(self):
        return _ptrs(self.bg) if self.bg is not None else None

    def advance(self, nsteps: int, t_end: float = 0.0) -> int:
        lib = _load()
        t = ctypes.c_double(self.t)
        done = ctypes.c_int(0)
        info = np.zeros(4)
        rc = lib.orc_advance(ctypes.byref(self.cfg), _ptrs(self.f), self._bgp(), int(nsteps),
                             float(t_end), ctypes.byref(t), ctypes.byref(done), info.ctypes.data_as(_P))
        self.t = t.value
        self.steps += done.value
        self.last = info
        if rc not in (OK, ENONPHYS):
            raise OracleError(rc, "orc_advance")
        return rc, done.value

    def advance_ext(self, nsteps: int, rext: np.ndarray, t_end: float = 0.0) -> int:
        """Advance with the coefficient ratios taken from rext (10, ny, nx) float32
        wherever a value is not negative (held fixed for the whole call)."""
        lib = _load()
        r = _f32_planes(rext, self.prob.nx, self.prob.ny)
        t = ctypes.c_double(self.t)
        done = ctypes.c_int(0)
        info = np.zeros(4)
        rc = lib.orc_advance_ext(ctypes.byref(self.cfg), _ptrs(self.f), int(nsteps), float(t_end),
                                 ctypes.byref(t), ctypes.byref(done), info.ctypes.data_as(_P),
                                 r.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        self.t = t.value
        self.steps += done.value
        self.last = info
        if rc != OK:
            raise OracleError(rc, "orc_advance_ext")
        return done.value

    def ratio_fields(self) -> np.ndarray:
        return ratio_fields(self.cfg, self.f, self.bg)

    def run(self, nsteps: int, t_end: float = 0.0) -> int:
        rc, done = self.advance(nsteps, t_end)
        if rc != OK:
            raise OracleError(rc, "orc_advance")
        return done

    def fields(self) -> Dict[str, np.ndarray]:
        return {k: a.copy() for k, a in zip(FIELDS, self.f)}

    def stacked(self) -> np.ndarray:
        return np.stack(self.f)

    def wavespeed(self):
        return wavespeed(self.cfg, self.f, self.bg)

    def rhs(self, cmax: Optional[float] = None) -> np.ndarray:
        if cmax is None:
            cmax = self.wavespeed()[2]
        return rhs(self.cfg, self.f, self.bg, cmax)

    def sums(self) -> np.ndarray:
        return sums(self.cfg, self.f)


def wavespeed(cfg: _Cfg, f: Sequence[np.ndarray], bg=None, check: bool = True):
    """(c_x, c_y, c_max, dt) of a state; raises OracleError on a non-physical state."""
    lib = _load()
    f = [_c64(a) for a in f]
    bgp = _ptrs([_c64(a) for a in bg]) if bg is not None else None
    out = np.zeros(4)
    rc = lib.orc_wavespeed(ctypes.byref(cfg), _ptrs(f), bgp, out.ctypes.data_as(_P))
    if rc != OK and check:
        raise OracleError(rc, "orc_wavespeed")
    return tuple(float(v) for v in out)


def rhs(cfg: _Cfg, f: Sequence[np.ndarray], bg, cmax: float) -> np.ndarray:
    lib = _load()
    f = [_c64(a) for a in f]
    bgp = _ptrs([_c64(a) for a in bg]) if bg is not None else None
    K = [np.zeros_like(f[0]) for _ in range(6)]
    rc = lib.orc_rhs(ctypes.byref(cfg), _ptrs(f), bgp, float(cmax), _ptrs(K))
    if rc != OK:
        raise OracleError(rc, "orc_rhs")
    return np.stack(K)


def step_patch(cfg: _Cfg, patch: Sequence[np.ndarray], bg_patch, dt: float, cmax: float) -> np.ndarray:
    """One RK4 step on a patch with a 12-cell supplied margin; returns (6, py-24, px-24)."""
    lib = _load()
    patch = [_c64(a) for a in patch]
    py, px = patch[0].shape
    bgp = _ptrs([_c64(a) for a in bg_patch]) if bg_patch is not None else None
    out = [np.zeros((py - 24, px - 24)) for _ in range(6)]
    rc = lib.orc_step_patch(ctypes.byref(cfg), px, py, _ptrs(patch), bgp, float(dt), float(cmax), _ptrs(out))
    if rc != OK:
        raise OracleError(rc, "orc_step_patch")
    return np.stack(out)


def _f32_planes(r, nx: int, ny: int) -> np.ndarray:
    r = np.ascontiguousarray(r, dtype=np.float32)
    if r.shape != (10, ny, nx):
        raise ValueError(f"ratio fields must have shape (10, {ny}, {nx}), got {r.shape}")
    return r


def rhs_ext(cfg: _Cfg, f: Sequence[np.ndarray], cmax: float, rext: np.ndarray) -> np.ndarray:
    """L(U) with externally supplied coefficient ratios (negative = plain)."""
    lib = _load()
    f = [_c64(a) for a in f]
    r = _f32_planes(rext, cfg.nx, cfg.ny)
    K = [np.zeros_like(f[0]) for _ in range(6)]
    rc = lib.orc_rhs_ext(ctypes.byref(cfg), _ptrs(f), float(cmax), _ptrs(K),
                         r.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    if rc != OK:
        raise OracleError(rc, "orc_rhs_ext")
    return np.stack(K)


def ratio_fields(cfg: _Cfg, f: Sequence[np.ndarray], bg=None) -> np.ndarray:
    """Plain coefficient ratios of every face: (10, ny, nx); planes 0-4 x faces
    {rho~, eps~, v_x, v_y, B~_y}, 5-9 y faces {rho~, eps~, v_x, v_y, B~_x}."""
    lib = _load()
    f = [_c64(a) for a in f]
    bgp = _ptrs([_c64(a) for a in bg]) if bg is not None else None
    out = np.zeros((10, cfg.ny, cfg.nx))
    rc = lib.orc_hd_ratio_fields(ctypes.byref(cfg), _ptrs(f), bgp, out.ctypes.data_as(_P))
    if rc != OK:
        raise OracleError(rc, "orc_hd_ratio_fields")
    return out


def face_fields(cfg: _Cfg, f: Sequence[np.ndarray], bg=None):
    """(R, D1): plain ratios and first differences of every face, each (10, ny, nx)."""
    lib = _load()
    f = [_c64(a) for a in f]
    bgp = _ptrs([_c64(a) for a in bg]) if bg is not None else None
    R = np.zeros((10, cfg.ny, cfg.nx))
    D1 = np.zeros((10, cfg.ny, cfg.nx))
    rc = lib.orc_hd_face_fields(ctypes.byref(cfg), _ptrs(f), bgp, R.ctypes.data_as(_P), D1.ctypes.data_as(_P))
    if rc != OK:
        raise OracleError(rc, "orc_hd_face_fields")
    return R, D1


def hd_check(cfg: _Cfg, f: Sequence[np.ndarray], rnn: np.ndarray, bound: float, tile: int, metric: int = 0):
    """Surrogate check: (mask (nty, ntx) of fallback tiles, n_fallback, err_used, err_all);
    metric 0 compares ratios, 1 the flux-weighted error."""
    lib = _load()
    f = [_c64(a) for a in f]
    r = _f32_planes(rnn, cfg.nx, cfg.ny)
    ntx, nty = -(-cfg.nx // tile), -(-cfg.ny // tile)
    mask = np.zeros((nty, ntx), dtype=np.int32)
    nf = ctypes.c_int(0)
    eu, ea = ctypes.c_double(0), ctypes.c_double(0)
    rc = lib.orc_hd_check(ctypes.byref(cfg), _ptrs(f), r.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                          float(bound), int(tile), int(metric), mask.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                          ctypes.byref(nf), ctypes.byref(eu), ctypes.byref(ea))
    if rc != OK:
        raise OracleError(rc, "orc_hd_check")
    return mask, nf.value, eu.value, ea.value


def sums(cfg: _Cfg, f: Sequence[np.ndarray]) -> np.ndarray:
    lib = _load()
    f = [_c64(a) for a in f]
    out = np.zeros(6)
    rc = lib.orc_sums(ctypes.byref(cfg), _ptrs(f), out.ctypes.data_as(_P))
    if rc != OK:
        raise OracleError(rc, "orc_sums")
    return out


def deriv_line(q: np.ndarray, h: float) -> np.ndarray:
    lib = _load()
    q = _c64(q)
    out = np.zeros_like(q)
    rc = lib.orc_deriv_line(q.size, q.ctypes.data_as(_P), float(h), out.ctypes.data_as(_P))
    if rc != OK:
        raise OracleError(rc, "orc_deriv_line")
    return out


def hd_ratio_line(q: np.ndarray) -> np.ndarray:
    """R on faces i+1/2 of a periodic line."""
    lib = _load()
    q = _c64(q)
    out = np.zeros_like(q)
    rc = lib.orc_hd_ratio_line(q.size, q.ctypes.data_as(_P), out.ctypes.data_as(_P))
    if rc != OK:
        raise OracleError(rc, "orc_hd_ratio_line")
    return out


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 (absolute when ||b|| = 0)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.sqrt(np.sum(b * b)))
    d = float(np.sqrt(np.sum((a - b) ** 2)))
    return d / nb if nb > 0 else d
