"""A domain split into px x py subdomains, one context each (paper section 3,
Fig. 1: the initial configuration divided into sub-regions, each advanced by
its own process with 'halo' layers exchanged through buffers before every
stage, and one time step for the whole domain).

Here every subdomain lives on the same GPU and stream, and the exchange is a
device buffer that one context packs and its neighbour unpacks; on several
GPUs the same buffers would travel between devices.  Each step takes the
wave-speed maxima over all subdomains (the step's only global reduction, a
device max here, an all-reduce(max) on several GPUs), then runs the four
stages, each after the x and then the y halo exchange.  The subdomains
evolve bit for bit as their parts of the undivided domain.
"""

from typing import List, Optional, Sequence

import ctypes

import torch

from .sacx import (EXCHANGE, FIELDS, FP64, OPEN, PERIODIC, Solver, StepGraph, _check, load_library, make_grid,
                   make_params, DEFAULT_C2, DEFAULT_CSHK)


def even_cuts(n: int, parts: int) -> List[int]:
    """Boundaries 0 = c_0 < ... < c_parts = n of parts near-equal pieces."""
    return [(n * k) // parts for k in range(parts + 1)]


class DecomposedSolver:
    """The subdomains of one problem and their exchange buffers."""

    def __init__(self, prob, xcuts: Sequence[int], ycuts: Sequence[int], precision=FP64, cfl=0.3, hd_on=True,
                 hd_cross_on=True, c2=DEFAULT_C2, cshk=DEFAULT_CSHK, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        if prob.background is not None:
            raise ValueError("exchange boundaries do not support a background")
        xcuts, ycuts = list(xcuts), list(ycuts)
        if xcuts[0] != 0 or xcuts[-1] != prob.nx or ycuts[0] != 0 or ycuts[-1] != prob.ny:
            raise ValueError("cuts must run from 0 to nx (ny)")
        self.prob, self.xcuts, self.ycuts = prob, xcuts, ycuts
        self.px, self.py = len(xcuts) - 1, len(ycuts) - 1
        dx = (prob.x1 - prob.x0) / prob.nx
        dy = (prob.y1 - prob.y0) / prob.ny
        params = make_params(prob.gamma, cfl, hd_on, hd_cross_on, c2, cshk, getattr(prob, "g", (0.0, 0.0)))
        self.subs: List[List[Solver]] = []
        for b in range(self.py):
            row = []
            for a in range(self.px):
                i0, i1, j0, j1 = xcuts[a], xcuts[a + 1], ycuts[b], ycuts[b + 1]
                grid = make_grid(i1 - i0, j1 - j0, prob.x0 + i0 * dx, prob.x0 + i1 * dx, prob.y0 + j0 * dy,
                                 prob.y0 + j1 * dy, precision, False)
                s = Solver(grid, params, self._sides(a, b), device=device, stream=stream)
                # the whole domain's spacing: the subdomain's extent over its
                # cell count can round differently
                s.set_spacing(dx, dy)
                f = torch.stack([torch.from_numpy(prob.fields[k][j0:j1, i0:i1].copy()) for k in FIELDS]).to(s.device)
                s.init_state(f, None, t0=prob.t0)
                row.append(s)
            self.subs.append(row)
        # every subdomain works on one stream, and so does the driver's own
        # device work (the maxima array)
        self.stream = self.subs[0][0].stream
        # the whole domain's wave-speed maxima, reduced on the device
        with torch.cuda.stream(self.stream):
            self.cmax = torch.zeros(2, dtype=torch.float64, device=self.subs[0][0].device)
        # buffers[b][a][side]: what subdomain (a, b) packs at `side` (the
        # Python-driven path)
        self.buffers = [[{side: s.halo_buffer(side) for side in range(4) if self._sides(a, b)[side] == EXCHANGE}
                         for a, s in enumerate(row)] for b, row in enumerate(self.subs)]
        # the library's own domain object (the native path): subdomain (a, b)
        # at a + b px, its strips and maxima in one caller-owned buffer
        self.lib = load_library()
        arr = (ctypes.c_void_p * (self.px * self.py))(*[s.ctx.value for row in self.subs for s in row])
        self._subs_arr = arr
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.sacx_domain_buffer_size(self.px, self.py, arr, ctypes.byref(nbytes)), "sacx_domain_buffer_size")
        with torch.cuda.stream(self.stream):
            self.domain_buf = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.subs[0][0].device)
        base = self.domain_buf.data_ptr()
        off = (-base) % 256
        self.domain = ctypes.c_void_p(None)
        _check(self.lib.sacx_domain_create(self.px, self.py, arr, ctypes.c_void_p(base + off), nbytes.value,
                                           ctypes.byref(self.domain)), "sacx_domain_create")

    def _sides(self, a: int, b: int):
        """Boundary kinds of subdomain (a, b): EXCHANGE towards a neighbour
        (the periodic image included), the domain's own kind otherwise."""
        bc = list(self.prob.bc)
        out = []
        for side in range(4):
            parts = self.px if side < 2 else self.py
            pos = a if side < 2 else b
            edge = (pos == 0) if side % 2 == 0 else (pos == parts - 1)
            if not edge:
                out.append(EXCHANGE)
            elif bc[side] == PERIODIC:
                out.append(EXCHANGE if parts > 1 else PERIODIC)
            else:
                out.append(OPEN)
        return tuple(out)

    def _neighbour(self, a: int, b: int, side: int):
        if side == 0:
            return (a - 1) % self.px, b
        if side == 1:
            return (a + 1) % self.px, b
        if side == 2:
            return a, (b - 1) % self.py
        return a, (b + 1) % self.py

    def _exchange(self, direction: int):
        sides = (0, 1) if direction == 0 else (2, 3)
        for b, row in enumerate(self.subs):
            for a, s in enumerate(row):
                for side in sides:
                    if side in self.buffers[b][a]:
                        s.halo_pack(side, self.buffers[b][a][side])
        for b, row in enumerate(self.subs):
            for a, s in enumerate(row):
                for side in sides:
                    if side in self.buffers[b][a]:
                        na, nb = self._neighbour(a, b, side)
                        s.halo_unpack(side, self.buffers[nb][na][side ^ 1])

    def wave_speeds(self):
        cx = cy = 0.0
        for row in self.subs:
            for s in row:
                x, y = s.wave_speeds()
                cx, cy = max(cx, x), max(cy, y)
        return cx, cy

    def advance(self, nsteps: int, device_max: bool = True, native: bool = True):
        """nsteps RK4 steps of the whole domain.  native: the library's domain
        object drives every launch (sacx_domain_advance); otherwise this class
        does, through the stage-level calls, with the maxima over the
        subdomains reduced on the device (device_max) or read back and
        reduced on the host."""
        if native and device_max:
            with torch.cuda.device(self.subs[0][0].device):
                _check(self.lib.sacx_domain_advance(self.domain, int(nsteps)), "sacx_domain_advance")
            return
        with torch.cuda.stream(self.stream):
            for _ in range(nsteps):
                self._step(device_max)

    def _step(self, device_max: bool):
        """Enqueue one step of the whole domain."""
        if device_max:
            self.cmax.zero_()
            for row in self.subs:
                for s in row:
                    s.wave_speeds_max(self.cmax)
            c = self.cmax
        else:
            c = self.wave_speeds()
        for _stage in range(4):
            for row in self.subs:
                for s in row:
                    s.fill_boundaries(0)
            self._exchange(0)
            for row in self.subs:
                for s in row:
                    s.fill_boundaries(1)
            self._exchange(1)
            for row in self.subs:
                for s in row:
                    s.stage(c)

    def graph(self, nsteps: int) -> StepGraph:
        """nsteps steps of the whole domain (the native path) captured into
        one HIP graph: every fill, pack, unpack, maximum and stage launch of
        every subdomain replayed as one graph launch.  Needs the subdomains
        on a stream of their own (DecomposedSolver(..., stream=...))."""
        return StepGraph(lambda: self.advance(nsteps), self.stream)

    def read_fields(self, dtype: torch.dtype = torch.float64) -> torch.Tensor:
        out = None
        for b, row in enumerate(self.subs):
            for a, s in enumerate(row):
                f = s.read_fields(dtype)
                if out is None:
                    out = torch.empty((6, self.prob.ny, self.prob.nx), dtype=dtype, device=f.device)
                out[:, self.ycuts[b]:self.ycuts[b + 1], self.xcuts[a]:self.xcuts[a + 1]] = f
        return out

    def diagnostics(self):
        return [[s.diagnostics() for s in row] for row in self.subs]

    def close(self):
        if getattr(self, "domain", None):
            self.lib.sacx_domain_destroy(self.domain)
            self.domain = ctypes.c_void_p(None)
        for row in self.subs:
            for s in row:
                s.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
