"""ctypes binding of the three-dimensional contexts of libsacx (include/sacx3.h).

Argument marshalling only: every step of the method runs in the HIP
library; PyTorch provides device memory (the caller-owned workspace and the
field buffers) and the stream.  No fallback: without the library every call
raises.
"""

from __future__ import annotations

import ctypes
from typing import Dict, Optional

import numpy as np
import torch

from . import sacx as _s

FIELDS3 = ("rho", "mx", "my", "mz", "e", "bx", "by", "bz")

EXPORTED3 = (
    "sacx3_workspace_size", "sacx3_create", "sacx3_destroy", "sacx3_set_boundaries", "sacx3_init_state",
    "sacx3_advance", "sacx3_read_fields", "sacx3_diagnostics", "sacx3_set_launch",
)


class Grid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("z0", ctypes.c_double), ("z1", ctypes.c_double)]


class Params3(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("hd_on", ctypes.c_int32), ("hd_cross_on", ctypes.c_int32),
                ("c2", ctypes.c_double * 4), ("cshk", ctypes.c_double * 4)]


class Diag3(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("c", ctypes.c_double * 3),
                ("c_max", ctypes.c_double), ("sums", ctypes.c_double * 8), ("steps", ctypes.c_int64),
                ("nonphys", ctypes.c_int32)]


_bound = False


def load_library():
    """libsacx.so with the 3-D entry points typed; raises if it is not built."""
    global _bound
    lib = _s.load_library()
    if not _bound:
        P = ctypes.c_void_p
        PP = ctypes.POINTER(ctypes.c_void_p)
        lib.sacx3_workspace_size.argtypes = [ctypes.POINTER(Grid3), ctypes.POINTER(Params3),
                                             ctypes.POINTER(ctypes.c_size_t)]
        lib.sacx3_create.argtypes = [ctypes.POINTER(Grid3), ctypes.POINTER(Params3), P, ctypes.c_size_t, P,
                                     ctypes.POINTER(P)]
        lib.sacx3_destroy.argtypes = [P]
        lib.sacx3_set_boundaries.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        lib.sacx3_init_state.argtypes = [P, PP, ctypes.c_int64, ctypes.c_int64, ctypes.c_double]
        lib.sacx3_advance.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_double)]
        lib.sacx3_read_fields.argtypes = [P, PP, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32]
        lib.sacx3_diagnostics.argtypes = [P, ctypes.POINTER(Diag3)]
        lib.sacx3_set_launch.argtypes = [P, ctypes.c_int32]
        for n in EXPORTED3:
            getattr(lib, n).restype = ctypes.c_int
        _bound = True
    return lib


def make_grid3(nx, ny, nz, extent) -> Grid3:
    e = [float(v) for v in extent]
    return Grid3(int(nx), int(ny), int(nz), *e)


def make_params3(gamma, cfl=0.3, hd_on=True, hd_cross_on=True, c2=_s.DEFAULT_C2, cshk=_s.DEFAULT_CSHK) -> Params3:
    return Params3(float(gamma), float(cfl), int(bool(hd_on)), int(bool(hd_cross_on)),
                   (ctypes.c_double * 4)(*c2), (ctypes.c_double * 4)(*cshk))


def workspace_size3(grid: Grid3, params: Params3) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    _s._check(lib.sacx3_workspace_size(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(n)),
              "sacx3_workspace_size")
    return n.value


class Solver3:
    """One three-dimensional context (sacx3_ctx) with its torch-owned workspace."""

    def __init__(self, grid: Grid3, params: Params3, bc=(_s.PERIODIC,) * 6, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        self.lib = load_library()
        self.grid, self.params = grid, params
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = workspace_size3(grid, params)
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _s._check(self.lib.sacx3_create(ctypes.byref(grid), ctypes.byref(params),
                                            ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.ctx)),
                      "sacx3_create")
        _s._live.add(self)
        self.set_boundaries(bc)

    @classmethod
    def from_problem(cls, prob, cfl=0.3, hd_on=True, hd_cross_on=True, c2=_s.DEFAULT_C2, cshk=_s.DEFAULT_CSHK,
                     device="cuda", init=True, **kw) -> "Solver3":
        grid = make_grid3(prob.nx, prob.ny, prob.nz, prob.extent)
        params = make_params3(prob.gamma, cfl, hd_on, hd_cross_on, c2, cshk)
        s = cls(grid, params, tuple(prob.bc), device=device, **kw)
        if init:
            f = torch.stack([torch.from_numpy(np.array(prob.fields[k], dtype=np.float64)) for k in FIELDS3]).to(s.device)
            s.init_state(f, t0=prob.t0)
        return s

    def close(self):
        """Destroy the context (its queued work finishes first)."""
        if self.ctx:
            with torch.cuda.device(self.device):
                self.lib.sacx3_destroy(self.ctx)
        self.ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shared(self):
        return _s.Solver._shared(self)

    def set_boundaries(self, bc):
        arr = (ctypes.c_int32 * 6)(*[int(b) for b in bc])
        _s._check(self.lib.sacx3_set_boundaries(self.ctx, arr), "sacx3_set_boundaries")

    def set_launch(self, planes: int):
        _s._check(self.lib.sacx3_set_launch(self.ctx, int(planes)), "sacx3_set_launch")

    def init_state(self, fields: torch.Tensor, t0: float = 0.0):
        """fields: (8, nz, ny, nx) float64 device tensor."""
        g = self.grid
        if fields.dim() != 4 or tuple(fields.shape) != (8, g.nz, g.ny, g.nx) or fields.device != self.device:
            raise ValueError(f"fields must be an (8, {g.nz}, {g.ny}, {g.nx}) tensor on {self.device}")
        if fields.dtype != torch.float64:
            raise ValueError("3-D fields are float64")
        fields = fields.contiguous()
        self._init_keep = fields
        with self._shared():
            _s._check(self.lib.sacx3_init_state(self.ctx, _s._ptrs([fields[k] for k in range(8)]), g.nx,
                                                g.nx * g.ny, float(t0)), "sacx3_init_state")

    def advance(self, nsteps: int, t_end: float = 0.0, sync: bool = True):
        """Enqueue nsteps; with sync, return (steps_done, t) and raise on a non-physical stop."""
        with torch.cuda.device(self.device):
            if not sync:
                _s._check(self.lib.sacx3_advance(self.ctx, int(nsteps), float(t_end), None, None), "sacx3_advance")
                return None
            done = ctypes.c_int32(0)
            t = ctypes.c_double(0.0)
            rc = self.lib.sacx3_advance(self.ctx, int(nsteps), float(t_end), ctypes.byref(done), ctypes.byref(t))
            _s._check(rc, "sacx3_advance")
            return done.value, t.value

    def advance_rc(self, nsteps: int, t_end: float = 0.0):
        """Like advance(sync=True) but return (rc, steps_done, t) instead of raising on ENONPHYS."""
        with torch.cuda.device(self.device):
            done = ctypes.c_int32(0)
            t = ctypes.c_double(0.0)
            rc = self.lib.sacx3_advance(self.ctx, int(nsteps), float(t_end), ctypes.byref(done), ctypes.byref(t))
            if rc not in (_s.OK, _s.ENONPHYS):
                _s._check(rc, "sacx3_advance")
            return rc, done.value, t.value

    def read_fields(self, mask: int = 0xFF) -> torch.Tensor:
        g = self.grid
        out = torch.zeros((8, g.nz, g.ny, g.nx), dtype=torch.float64, device=self.device)
        with self._shared():
            _s._check(self.lib.sacx3_read_fields(self.ctx, _s._ptrs([out[k] for k in range(8)]), g.nx, g.nx * g.ny,
                                                 int(mask)), "sacx3_read_fields")
        return out

    def diagnostics(self) -> Dict:
        d = Diag3()
        with torch.cuda.device(self.device):
            _s._check(self.lib.sacx3_diagnostics(self.ctx, ctypes.byref(d)), "sacx3_diagnostics")
        return {"t": d.t, "dt": d.dt, "c": list(d.c), "c_max": d.c_max, "sums": list(d.sums), "steps": d.steps,
                "nonphys": d.nonphys}
