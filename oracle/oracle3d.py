"""FP64 CPU oracle of the scheme in three dimensions -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` and the CPU-baseline leg of ``bench.py`` may import this
module.  The C source ``sacx_oracle3d.c`` is built with gcc -O2
-ffp-contract=off and driven through ctypes; it shares no code with the GPU
library.  Inputs come from ``workloads`` (Problem3).

Parity status: pinned by the CPU tests to the (pinned) 2-D oracle bit for
bit in all three planes, and to closed forms and invariants in 3-D (uniform
states, the oblique entropy wave's order, conservation, div B, axis
permutations).  The hyper-diffusion constants remain "parity unpinned", as
in two dimensions.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sacx_oracle3d.c")
_LIB = os.environ.get("SACX_ORACLE3D_LIB") or os.path.join(_HERE, "libsacx_oracle3d.so")

FIELDS3 = ("rho", "mx", "my", "mz", "e", "bx", "by", "bz")
OK, EINVAL, ENONPHYS, ENOMEM = 0, -1, -4, -7
PERIODIC, OPEN = 0, 1
PAPER, LOWSTORE = 0, 1
DEFAULT_C2 = (0.02, 0.02, 0.2, 0.02)
DEFAULT_CSHK = (0.5, 0.5, 0.5, 0.5)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                        "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Cfg3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("z0", ctypes.c_double), ("z1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("hd_on", ctypes.c_int), ("hd_cross_on", ctypes.c_int),
        ("c2", ctypes.c_double * 4), ("cshk", ctypes.c_double * 4),
        ("bc", ctypes.c_int * 6),
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
            C = ctypes.POINTER(Cfg3)
            lib.orc3_advance.argtypes = [C, _PP, ctypes.c_int, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_int), _P]
            lib.orc3_rhs.argtypes = [C, _PP, ctypes.c_double, _PP]
            lib.orc3_wavespeed.argtypes = [C, _PP, _P]
            lib.orc3_sums.argtypes = [C, _PP, _P]
            for n in ("orc3_advance", "orc3_rhs", "orc3_wavespeed", "orc3_sums", "orc3_abi_version"):
                getattr(lib, n).restype = ctypes.c_int
            _lib = lib
    return _lib


def make_cfg(prob, cfl: float = 0.3, hd_on: bool = True, hd_cross_on: bool = True, c2=DEFAULT_C2,
             cshk=DEFAULT_CSHK, form: int = PAPER) -> Cfg3:
    e = prob.extent
    return Cfg3(prob.nx, prob.ny, prob.nz, e[0], e[1], e[2], e[3], e[4], e[5], prob.gamma, cfl, int(hd_on),
                int(hd_cross_on), (ctypes.c_double * 4)(*c2), (ctypes.c_double * 4)(*cshk),
                (ctypes.c_int * 6)(*prob.bc), int(form))


def _fields_ptrs(arr: np.ndarray):
    arrs = [np.ascontiguousarray(arr[k]) for k in range(8)]
    ptrs = (_P * 8)(*[a.ctypes.data_as(_P) for a in arrs])
    return arrs, ptrs


class State3:
    """A 3-D state advanced by the oracle (fields (8, nz, ny, nx) float64)."""

    def __init__(self, prob, form: int = PAPER, **kw):
        self.prob = prob
        self.cfg = make_cfg(prob, form=form, **kw)
        self.f = prob.stacked()
        self.t = float(prob.t0)
        self.steps = 0
        self.info = np.zeros(5)

    def run(self, nsteps: int, t_end: float = 0.0) -> int:
        lib = _load()
        arrs, ptrs = _fields_ptrs(self.f)
        t = ctypes.c_double(self.t)
        done = ctypes.c_int(0)
        info = np.zeros(5)
        rc = lib.orc3_advance(ctypes.byref(self.cfg), ptrs, int(nsteps), float(t_end), ctypes.byref(t),
                              ctypes.byref(done), info.ctypes.data_as(_P))
        self.f = np.stack(arrs)
        self.t = t.value
        self.steps += done.value
        self.info = info
        if rc not in (OK, ENONPHYS):
            raise RuntimeError(f"orc3_advance failed ({rc})")
        return rc

    def sums(self) -> np.ndarray:
        return sums(self.cfg, self.f)


def rhs(cfg: Cfg3, f: np.ndarray, cmax: float) -> np.ndarray:
    lib = _load()
    arrs, ptrs = _fields_ptrs(f)
    out = np.zeros_like(f)
    outs = [np.ascontiguousarray(out[k]) for k in range(8)]
    optr = (_P * 8)(*[a.ctypes.data_as(_P) for a in outs])
    rc = lib.orc3_rhs(ctypes.byref(cfg), ptrs, float(cmax), optr)
    if rc:
        raise RuntimeError(f"orc3_rhs failed ({rc})")
    return np.stack(outs)


def wavespeed(cfg: Cfg3, f: np.ndarray):
    """(c_x, c_y, c_z, c_max, dt) of a state; raises on a non-physical one."""
    lib = _load()
    arrs, ptrs = _fields_ptrs(f)
    out = np.zeros(5)
    rc = lib.orc3_wavespeed(ctypes.byref(cfg), ptrs, out.ctypes.data_as(_P))
    if rc:
        raise RuntimeError(f"orc3_wavespeed: non-physical or invalid ({rc})")
    return tuple(float(v) for v in out)


def sums(cfg: Cfg3, f: np.ndarray) -> np.ndarray:
    lib = _load()
    arrs, ptrs = _fields_ptrs(f)
    out = np.zeros(8)
    rc = lib.orc3_sums(ctypes.byref(cfg), ptrs, out.ctypes.data_as(_P))
    if rc:
        raise RuntimeError(f"orc3_sums failed ({rc})")
    return out
