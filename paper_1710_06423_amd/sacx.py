"""ctypes binding of libsacx (the C ABI declared in include/sacx.h).

Argument marshalling only: every step of the method runs in the HIP
library; PyTorch provides device memory (the caller-owned workspace and
field buffers) and the stream.  If the library is not built the import of
this module succeeds but every call raises -- there is no fallback path.
"""

from __future__ import annotations

import atexit
import contextlib
import ctypes
import os
import weakref
from typing import Dict, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsacx.so")

OK, EINVAL, ENOSPC, EDEVICE, ENONPHYS, EUNSUP, ESTATE = 0, -1, -2, -3, -4, -5, -6
PERIODIC, OPEN, EXCHANGE = 0, 1, 2
PROBLEM_ORSZAG_TANG, PROBLEM_BRIO_WU = 0, 1
FP64, FP32 = 0, 1
GHOST = 3
FIELDS = ("rho", "mx", "my", "e", "bx", "by")
BACKGROUND_FIELDS = ("rho_b", "e_b", "bx_b", "by_b")

# Hyper-diffusion constants (density, thermal energy, velocity, field): the
# scheme's frozen defaults; the paper gives no values.
DEFAULT_C2 = (0.02, 0.02, 0.2, 0.02)
DEFAULT_CSHK = (0.5, 0.5, 0.5, 0.5)

EXPORTED = (
    "sacx_abi_version", "sacx_strerror", "sacx_last_error", "sacx_workspace_size", "sacx_create",
    "sacx_destroy", "sacx_set_boundaries", "sacx_init_state", "sacx_init_problem", "sacx_advance", "sacx_read_fields",
    "sacx_diagnostics", "sacx_halo_buffer_size", "sacx_halo_pack", "sacx_halo_unpack",
    "sacx_fill_boundaries", "sacx_stage", "sacx_wave_speeds", "sacx_wave_speeds_max", "sacx_set_spacing",
    "sacx_domain_buffer_size", "sacx_domain_create", "sacx_domain_advance", "sacx_domain_destroy",
    "sacx_profile_enable", "sacx_profile_read", "sacx_set_launch", "sacx_get_launch", "sacx_set_column_split",
    "sacx_batch_workspace_size", "sacx_batch_create", "sacx_batch_destroy", "sacx_batch_context",
    "sacx_batch_set_tiles", "sacx_batch_advance",
    "sacx_cnn_buffer_sizes", "sacx_cnn_pack", "sacx_cnn_forward", "sacx_cnn_backward",
    "sacx_cnn_backward_noalloc", "sacx_cnn_adam",
    "sacx_cnn_inputs", "sacx_hd_ratio_fields", "sacx_surrogate_workspace_size", "sacx_hd_set_surrogate",
    "sacx_hd_clear_surrogate", "sacx_hd_ratio_buffer", "sacx_hd_read_stats",
)

CNN_NPARAM = 23146
CNN_PACKED_BYTES = 99840
CNN_STATIC_WORK_BYTES = 64 << 20


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("precision", ctypes.c_int32), ("background_on", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("hd_on", ctypes.c_int32), ("hd_cross_on", ctypes.c_int32),
                ("c2", ctypes.c_double * 4), ("cshk", ctypes.c_double * 4), ("g", ctypes.c_double * 2)]


class Diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double),
                ("c_x", ctypes.c_double), ("c_y", ctypes.c_double), ("c_max", ctypes.c_double),
                ("sums", ctypes.c_double * 6), ("steps", ctypes.c_int64), ("nonphys", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("ms_stage", ctypes.c_double * 4), ("ms_halo", ctypes.c_double), ("ms_scalar", ctypes.c_double),
                ("n_stage", ctypes.c_int64 * 4), ("n_halo", ctypes.c_int64), ("n_scalar", ctypes.c_int64),
                ("ms_surrogate", ctypes.c_double), ("n_surrogate", ctypes.c_int64)]


class CnnSizes(ctypes.Structure):
    _fields_ = [("input_bytes", ctypes.c_size_t), ("act_bytes", ctypes.c_size_t),
                ("out_bytes", ctypes.c_size_t), ("work_bytes", ctypes.c_size_t)]


CHECK_RATIO, CHECK_FLUX = 0, 1


class Surrogate(ctypes.Structure):
    _fields_ = [("d_packed", ctypes.c_void_p), ("norm", ctypes.c_float * 12), ("refresh_every", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("metric", ctypes.c_int32), ("bound", ctypes.c_double)]


class HdStats(ctypes.Structure):
    _fields_ = [("refreshes", ctypes.c_int64), ("tiles_checked", ctypes.c_int64),
                ("tiles_fallback", ctypes.c_int64), ("err_used", ctypes.c_double), ("err_all", ctypes.c_double)]


class SacxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


_lib = None

# Contexts and batches still open: closed at interpreter exit, while the HIP
# runtime is still up (Python's exit handlers run before the C library's),
# so no library handle is released during the runtime's own teardown.
_live = weakref.WeakSet()


@atexit.register
def _close_live():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def load_library():
    """Load libsacx.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1710_06423_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.sacx_abi_version.restype = ctypes.c_int
    lib.sacx_strerror.restype = ctypes.c_char_p
    lib.sacx_strerror.argtypes = [ctypes.c_int]
    lib.sacx_last_error.restype = ctypes.c_char_p
    lib.sacx_workspace_size.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]
    lib.sacx_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Params), P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    lib.sacx_destroy.argtypes = [P]
    lib.sacx_set_boundaries.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    lib.sacx_init_state.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_double]
    lib.sacx_init_problem.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                      ctypes.c_double]
    lib.sacx_advance.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double)]
    lib.sacx_read_fields.argtypes = [P, ctypes.POINTER(P), ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32]
    lib.sacx_diagnostics.argtypes = [P, ctypes.POINTER(Diag)]
    lib.sacx_halo_buffer_size.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    lib.sacx_halo_pack.argtypes = [P, ctypes.c_int32, P]
    lib.sacx_halo_unpack.argtypes = [P, ctypes.c_int32, P]
    lib.sacx_fill_boundaries.argtypes = [P, ctypes.c_int32]
    lib.sacx_stage.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.sacx_wave_speeds_max.argtypes = [P, P]
    lib.sacx_domain_buffer_size.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)]
    lib.sacx_domain_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(P), P, ctypes.c_size_t,
                                       ctypes.POINTER(P)]
    lib.sacx_domain_advance.argtypes = [P, ctypes.c_int32]
    lib.sacx_domain_destroy.argtypes = [P]
    lib.sacx_wave_speeds.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.sacx_set_spacing.argtypes = [P, ctypes.c_double, ctypes.c_double]
    lib.sacx_profile_enable.argtypes = [P, ctypes.c_int32]
    lib.sacx_profile_read.argtypes = [P, ctypes.POINTER(Profile)]
    lib.sacx_set_launch.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.sacx_get_launch.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.sacx_set_column_split.argtypes = [P, ctypes.c_int32]
    lib.sacx_batch_workspace_size.argtypes = [ctypes.c_int32, ctypes.POINTER(Grid), ctypes.POINTER(Params),
                                              ctypes.POINTER(ctypes.c_size_t)]
    lib.sacx_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(Grid), ctypes.POINTER(Params),
                                      ctypes.POINTER(ctypes.c_int32), P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    lib.sacx_batch_destroy.argtypes = [P]
    lib.sacx_batch_context.argtypes = [P, ctypes.c_int32, ctypes.POINTER(P)]
    lib.sacx_batch_set_tiles.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.sacx_batch_advance.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    I32, SZ = ctypes.c_int32, ctypes.c_size_t
    lib.sacx_cnn_buffer_sizes.argtypes = [I32, I32, I32, ctypes.POINTER(CnnSizes)]
    lib.sacx_cnn_pack.argtypes = [P, P, P]
    lib.sacx_cnn_forward.argtypes = [P, P, I32, I32, I32, P, P, P]
    lib.sacx_cnn_backward.argtypes = [P, P, P, P, P, P, I32, I32, I32, P, SZ, P, P, P]
    lib.sacx_cnn_backward_noalloc.argtypes = [P, P, P, P, P, P, I32, I32, I32, P, P, P]
    lib.sacx_cnn_adam.argtypes = [P, P, P, P, I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, P]
    lib.sacx_cnn_inputs.argtypes = [P, ctypes.POINTER(ctypes.c_float), P]
    lib.sacx_hd_ratio_fields.argtypes = [P, P, P, ctypes.c_int64]
    lib.sacx_surrogate_workspace_size.argtypes = [P, ctypes.POINTER(SZ)]
    lib.sacx_hd_set_surrogate.argtypes = [P, ctypes.POINTER(Surrogate), P, SZ]
    lib.sacx_hd_clear_surrogate.argtypes = [P]
    lib.sacx_hd_ratio_buffer.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64)]
    lib.sacx_hd_read_stats.argtypes = [P, ctypes.POINTER(HdStats)]
    for n in EXPORTED:
        if n not in ("sacx_strerror", "sacx_last_error"):
            getattr(lib, n).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != OK:
        lib = load_library()
        msg = lib.sacx_last_error().decode() or lib.sacx_strerror(rc).decode()
        raise SacxError(rc, f"{what}: {msg} (code {rc})")


def make_grid(nx, ny, x0, x1, y0, y1, precision=FP64, background_on=False) -> Grid:
    return Grid(int(nx), int(ny), float(x0), float(x1), float(y0), float(y1), int(precision), int(bool(background_on)))


def make_params(gamma, cfl=0.3, hd_on=True, hd_cross_on=True, c2=DEFAULT_C2, cshk=DEFAULT_CSHK,
                g=(0.0, 0.0)) -> Params:
    return Params(float(gamma), float(cfl), int(bool(hd_on)), int(bool(hd_cross_on)),
                  (ctypes.c_double * 4)(*c2), (ctypes.c_double * 4)(*cshk), (ctypes.c_double * 2)(*g))


def workspace_size(grid: Grid, params: Params) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.sacx_workspace_size(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(n)), "sacx_workspace_size")
    return n.value


def _ptrs(tensors: Sequence[Optional[torch.Tensor]]):
    arr = (ctypes.c_void_p * len(tensors))()
    for k, t in enumerate(tensors):
        arr[k] = None if t is None else t.data_ptr()
    return arr


class Solver:
    """One subdomain context (sacx_ctx) with its torch-owned workspace."""

    def __init__(self, grid: Grid, params: Params, bc=(PERIODIC,) * 4, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None, _borrow=None):
        self.lib = load_library()
        self.owned = _borrow is None
        self.grid, self.params = grid, params
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.dtype = torch.float64 if grid.precision == FP64 else torch.float32
        if _borrow is not None:
            self.workspace = None
            self.ctx = _borrow
            return
        nbytes = workspace_size(grid, params)
        # allocated on the context's stream: the caching allocator hands the
        # block back to that stream's pool when it is freed, so a later
        # allocation there is ordered after the context's queued kernels
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(self.lib.sacx_create(ctypes.byref(grid), ctypes.byref(params),
                                        ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.ctx)),
                   "sacx_create")
        _live.add(self)
        self.set_boundaries(bc)
        self.dtype = torch.float64 if grid.precision == FP64 else torch.float32

    @classmethod
    def from_problem(cls, prob, precision=FP64, cfl=0.3, hd_on=True, hd_cross_on=True, c2=DEFAULT_C2,
                     cshk=DEFAULT_CSHK, device="cuda", init=True, **kw) -> "Solver":
        grid = make_grid(prob.nx, prob.ny, prob.x0, prob.x1, prob.y0, prob.y1, precision,
                         prob.background is not None)
        params = make_params(prob.gamma, cfl, hd_on, hd_cross_on, c2, cshk, getattr(prob, "g", (0.0, 0.0)))
        s = cls(grid, params, tuple(prob.bc), device=device, **kw)
        if init:
            f = torch.stack([torch.from_numpy(prob.fields[k]) for k in FIELDS]).to(s.device)
            bg = None
            if prob.background is not None:
                bg = torch.stack([torch.from_numpy(prob.background[k]) for k in BACKGROUND_FIELDS]).to(s.device)
            s.init_state(f, bg, t0=prob.t0)
        return s

    def close(self):
        """Destroy the context; its queued work finishes first (sacx_destroy
        waits for the stream), then the workspace can be freed."""
        if self.ctx and self.owned:
            with torch.cuda.device(self.device):
                self.lib.sacx_destroy(self.ctx)
        self.ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @contextlib.contextmanager
    def _shared(self):
        """Order the device tensors a call shares with the library when the
        caller's current stream is not the context's: the context's stream
        first waits for the caller's (inputs it produced, outputs it just
        allocated and cleared), and the caller's stream then waits for the
        context's (results it will read).  The tensors stay the caller's."""
        cur = torch.cuda.current_stream(self.device)
        same = cur.cuda_stream == self.stream.cuda_stream
        if not same:
            self.stream.wait_stream(cur)
        try:
            with torch.cuda.device(self.device):
                yield
        finally:
            # also when the call failed: it may have enqueued work before
            # returning its error
            if not same:
                cur.wait_stream(self.stream)

    def set_boundaries(self, bc):
        arr = (ctypes.c_int32 * 4)(*[int(b) for b in bc])
        _check(self.lib.sacx_set_boundaries(self.ctx, arr), "sacx_set_boundaries")

    def init_state(self, fields: torch.Tensor, bg: Optional[torch.Tensor] = None, t0: float = 0.0):
        """fields: (6, ny, nx) float64/float32 device tensor (rows contiguous)."""
        if fields.dim() != 3 or fields.shape[0] != 6 or fields.device != self.device:
            raise ValueError(f"fields must be a (6, ny, nx) tensor on {self.device}, got {tuple(fields.shape)} on {fields.device}")
        if fields.shape[1] != self.grid.ny or fields.shape[2] != self.grid.nx:
            raise ValueError("fields shape does not match the grid")
        fields = fields.contiguous()
        prec = FP64 if fields.dtype == torch.float64 else FP32
        self._init_keep = (fields, bg)
        bgp = None
        if bg is not None:
            bg = bg.to(fields.dtype).contiguous()
            bgp = _ptrs([bg[k] for k in range(4)])
        with self._shared():
            _check(self.lib.sacx_init_state(self.ctx, _ptrs([fields[k] for k in range(6)]), bgp,
                                            fields.shape[2], prec, float(t0)), "sacx_init_state")

    def init_problem(self, kind: int, prm: Sequence[float] = (), t0: float = 0.0):
        """Generate a verification problem on the device (sacx_init_problem):
        PROBLEM_ORSZAG_TANG (prm: B0 scale) or PROBLEM_BRIO_WU (prm: left and
        right scale); sets that problem's boundaries."""
        arr = (ctypes.c_double * max(len(prm), 1))(*[float(v) for v in prm])
        with torch.cuda.device(self.device):
            _check(self.lib.sacx_init_problem(self.ctx, int(kind), arr, len(prm), float(t0)), "sacx_init_problem")

    def advance(self, nsteps: int, t_end: float = 0.0, sync: bool = True):
        """Enqueue nsteps; with sync, return (steps_done, t) and raise on a non-physical stop."""
        with torch.cuda.device(self.device):
            if not sync:
                _check(self.lib.sacx_advance(self.ctx, int(nsteps), float(t_end), None, None), "sacx_advance")
                return None
            done = ctypes.c_int32(0)
            t = ctypes.c_double(0.0)
            rc = self.lib.sacx_advance(self.ctx, int(nsteps), float(t_end), ctypes.byref(done), ctypes.byref(t))
            self.last_rc = rc
            _check(rc, "sacx_advance")
            return done.value, t.value

    def advance_rc(self, nsteps: int, t_end: float = 0.0):
        """Like advance(sync=True) but return (rc, steps_done, t) instead of raising on ENONPHYS."""
        with torch.cuda.device(self.device):
            done = ctypes.c_int32(0)
            t = ctypes.c_double(0.0)
            rc = self.lib.sacx_advance(self.ctx, int(nsteps), float(t_end), ctypes.byref(done), ctypes.byref(t))
            if rc not in (OK, ENONPHYS):
                _check(rc, "sacx_advance")
            return rc, done.value, t.value

    def read_fields(self, dtype: torch.dtype = torch.float64, mask: int = 0x3F) -> torch.Tensor:
        out = torch.zeros((6, self.grid.ny, self.grid.nx), dtype=dtype, device=self.device)
        prec = FP64 if dtype == torch.float64 else FP32
        with self._shared():
            _check(self.lib.sacx_read_fields(self.ctx, _ptrs([out[k] for k in range(6)]), self.grid.nx, mask, prec),
                   "sacx_read_fields")
        return out

    def diagnostics(self) -> Dict:
        d = Diag()
        with torch.cuda.device(self.device):
            _check(self.lib.sacx_diagnostics(self.ctx, ctypes.byref(d)), "sacx_diagnostics")
        return {"t": d.t, "dt": d.dt, "c_x": d.c_x, "c_y": d.c_y, "c_max": d.c_max,
                "sums": list(d.sums), "steps": d.steps, "nonphys": d.nonphys}

    def halo_buffer(self, side: int) -> torch.Tensor:
        n = ctypes.c_size_t(0)
        _check(self.lib.sacx_halo_buffer_size(self.ctx, int(side), ctypes.byref(n)), "sacx_halo_buffer_size")
        buf = torch.zeros(n.value // (8 if self.grid.precision == FP64 else 4), dtype=self.dtype,
                          device=self.device)
        # the context's stream uses it too: its block is not reused before
        # the work queued there when it is freed has finished
        buf.record_stream(self.stream)
        return buf

    def halo_pack(self, side: int, buf: torch.Tensor):
        with self._shared():
            _check(self.lib.sacx_halo_pack(self.ctx, int(side), ctypes.c_void_p(buf.data_ptr())), "sacx_halo_pack")

    def halo_unpack(self, side: int, buf: torch.Tensor):
        with self._shared():
            _check(self.lib.sacx_halo_unpack(self.ctx, int(side), ctypes.c_void_p(buf.data_ptr())), "sacx_halo_unpack")

    def fill_boundaries(self, direction: int):
        """Fill the PERIODIC / OPEN ghost cells of one direction (0: x, 1: y)
        of the state the next stage differences."""
        with torch.cuda.device(self.device):
            _check(self.lib.sacx_fill_boundaries(self.ctx, int(direction)), "sacx_fill_boundaries")

    def stage(self, c_max=None) -> int:
        """Enqueue the next RK4 stage; c_max (x, y) is the whole domain's
        wave-speed maxima, used when the stage begins a step: a pair of
        floats, or a float64 device tensor of 2 elements read on the stream."""
        done = ctypes.c_int32(0)
        if isinstance(c_max, torch.Tensor):
            if c_max.dtype != torch.float64 or c_max.numel() != 2 or c_max.device != self.device:
                raise ValueError(f"c_max must be 2 float64 values on {self.device}")
            c, on_dev = ctypes.c_void_p(c_max.data_ptr()), 1
        elif c_max is None:
            c, on_dev = None, 0
        else:
            arr = (ctypes.c_double * 2)(*[float(v) for v in c_max])
            c, on_dev = ctypes.cast(arr, ctypes.c_void_p), 0
        with self._shared():
            _check(self.lib.sacx_stage(self.ctx, c, on_dev, ctypes.byref(done)), "sacx_stage")
        return done.value

    def wave_speeds_max(self, c_max: torch.Tensor):
        """Enqueue c_max = max(c_max, this context's maxima) on a float64
        device tensor of 2 elements."""
        if c_max.dtype != torch.float64 or c_max.numel() != 2 or c_max.device != self.device:
            raise ValueError(f"c_max must be 2 float64 values on {self.device}")
        with self._shared():
            _check(self.lib.sacx_wave_speeds_max(self.ctx, ctypes.c_void_p(c_max.data_ptr())), "sacx_wave_speeds_max")

    def set_spacing(self, dx: float, dy: float):
        """Grid spacing in place of the extent over the cell count (a
        subdomain takes the whole domain's)."""
        _check(self.lib.sacx_set_spacing(self.ctx, float(dx), float(dy)), "sacx_set_spacing")

    def wave_speeds(self):
        """(c_x, c_y) maxima of the current state's interior (synchronises)."""
        c = (ctypes.c_double * 2)()
        with torch.cuda.device(self.device):
            _check(self.lib.sacx_wave_speeds(self.ctx, c), "sacx_wave_speeds")
        return c[0], c[1]

    def profile_enable(self, on: bool = True):
        _check(self.lib.sacx_profile_enable(self.ctx, int(bool(on))), "sacx_profile_enable")
        self._profiling = bool(on)

    def graph(self, nsteps: int) -> "StepGraph":
        """nsteps RK4 steps captured into a HIP graph; each replay advances
        the state by nsteps as advance(nsteps, sync=False) would.  Needs a
        context on its own stream (Solver(..., stream=torch.cuda.Stream()))
        and profiling off; without a learned coefficient, whose refresh
        schedule lives on the host."""
        if getattr(self, "_profiling", False):
            raise ValueError("turn profiling off before capturing")
        if getattr(self, "sur_ws", None) is not None:
            raise ValueError("a context with a learned coefficient cannot be captured")
        return StepGraph(lambda: self.advance(nsteps, sync=False), self.stream)

    def profile_read(self) -> Dict:
        p = Profile()
        with torch.cuda.device(self.device):
            _check(self.lib.sacx_profile_read(self.ctx, ctypes.byref(p)), "sacx_profile_read")
        return {"ms_stage": list(p.ms_stage), "n_stage": list(p.n_stage), "ms_halo": p.ms_halo,
                "n_halo": p.n_halo, "ms_scalar": p.ms_scalar, "n_scalar": p.n_scalar,
                "ms_surrogate": p.ms_surrogate, "n_surrogate": p.n_surrogate}

    # ------------------------------------------------ learned coefficient
    def cnn_inputs(self, norm: Sequence[float], out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Network input image of the current state: (ny, nx, 8) BF16 (as int16 storage)."""
        if out is None:
            out = torch.empty((self.grid.ny, self.grid.nx, 8), dtype=torch.bfloat16, device=self.device)
        arr = (ctypes.c_float * 12)(*[float(v) for v in norm])
        with self._shared():
            _check(self.lib.sacx_cnn_inputs(self.ctx, arr, ctypes.c_void_p(out.data_ptr())), "sacx_cnn_inputs")
        return out

    def ratio_fields(self, out: Optional[torch.Tensor] = None, with_d1: bool = False):
        """Plain coefficient ratios of the current state: (10, ny, nx) float32
        (and the face first differences, same shape, with with_d1)."""
        shape = (10, self.grid.ny, self.grid.nx)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        d1 = torch.empty(shape, dtype=torch.float32, device=self.device) if with_d1 else None
        with self._shared():
            _check(self.lib.sacx_hd_ratio_fields(self.ctx, ctypes.c_void_p(out.data_ptr()),
                                                 ctypes.c_void_p(None if d1 is None else d1.data_ptr()),
                                                 self.grid.nx), "sacx_hd_ratio_fields")
        return (out, d1) if with_d1 else out

    def set_surrogate(self, packed: Optional[torch.Tensor], norm: Sequence[float], refresh_every: int = 1,
                      tile: int = 32, bound: float = 0.05, metric: int = CHECK_FLUX):
        """Switch the learned coefficient on (packed=None: the caller writes ratio_buffer())."""
        n = ctypes.c_size_t(0)
        _check(self.lib.sacx_surrogate_workspace_size(self.ctx, ctypes.byref(n)), "sacx_surrogate_workspace_size")
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            self.sur_ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self.sur_packed = packed
        cfg = Surrogate(None if packed is None else packed.data_ptr(), (ctypes.c_float * 12)(*[float(v) for v in norm]),
                        int(refresh_every), int(tile), int(metric), float(bound))
        with self._shared():
            _check(self.lib.sacx_hd_set_surrogate(self.ctx, ctypes.byref(cfg), ctypes.c_void_p(self.sur_ws.data_ptr()),
                                                  n.value), "sacx_hd_set_surrogate")

    def clear_surrogate(self):
        _check(self.lib.sacx_hd_clear_surrogate(self.ctx), "sacx_hd_clear_surrogate")
        self.sur_ws = None
        self.sur_packed = None

    def ratio_buffer(self) -> torch.Tensor:
        """The surrogate's ratio planes as a (10, ny, nx) float32 view (writable)."""
        ptr = ctypes.c_void_p(None)
        pitch = ctypes.c_int64(0)
        _check(self.lib.sacx_hd_ratio_buffer(self.ctx, ctypes.byref(ptr), ctypes.byref(pitch)), "sacx_hd_ratio_buffer")
        off = ptr.value - self.sur_ws.data_ptr()
        ny, nx, p = self.grid.ny, self.grid.nx, pitch.value
        flat = self.sur_ws[off: off + 10 * p * ny * 4].view(torch.float32)
        return flat.view(10, ny, p)[:, :, :nx]

    def hd_stats(self) -> Dict:
        st = HdStats()
        with torch.cuda.device(self.device):
            _check(self.lib.sacx_hd_read_stats(self.ctx, ctypes.byref(st)), "sacx_hd_read_stats")
        return {"refreshes": st.refreshes, "tiles_checked": st.tiles_checked, "tiles_fallback": st.tiles_fallback,
                "err_used": st.err_used, "err_all": st.err_all}

    def set_launch(self, threads: int = 0, rows: int = 0):
        _check(self.lib.sacx_set_launch(self.ctx, int(threads), int(rows)), "sacx_set_launch")

    def set_column_split(self, on: bool):
        """Two threads per column (x and y roles) for FP64 hyper-diffusion
        tiles (default), or one; bit-identical results."""
        _check(self.lib.sacx_set_column_split(self.ctx, int(bool(on))), "sacx_set_column_split")

    def get_launch(self):
        t, r = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(self.lib.sacx_get_launch(self.ctx, ctypes.byref(t), ctypes.byref(r)), "sacx_get_launch")
        return t.value, r.value


class Batch:
    """Many independent subdomains advanced by one persistent launch
    (sacx_batch_*).  Instance i is a borrowed context: ``batch[i]`` is a
    Solver view of it (init_state / read_fields / diagnostics / advance)."""

    def __init__(self, problems, precision=FP32, cfl=0.3, c2=DEFAULT_C2, cshk=DEFAULT_CSHK, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None, init=True):
        self.lib = load_library()
        n = len(problems)
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.grids = (Grid * n)(*[make_grid(p.nx, p.ny, p.x0, p.x1, p.y0, p.y1, precision, False) for p in problems])
        self.params = (Params * n)(*[make_params(p.gamma, cfl, True, True, c2, cshk, getattr(p, "g", (0.0, 0.0)))
                                     for p in problems])
        bc = (ctypes.c_int32 * (4 * n))(*[int(b) for p in problems for b in p.bc])
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.sacx_batch_workspace_size(n, self.grids, self.params, ctypes.byref(nbytes)),
               "sacx_batch_workspace_size")
        with torch.cuda.device(dev), torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        with torch.cuda.device(dev):
            self.b = ctypes.c_void_p(None)
            _check(self.lib.sacx_batch_create(n, self.grids, self.params, bc, ctypes.c_void_p(self.workspace.data_ptr()),
                                              nbytes.value, ctypes.c_void_p(self.stream.cuda_stream),
                                              ctypes.byref(self.b)), "sacx_batch_create")
        _live.add(self)
        self.n = n
        self.views = []
        for i in range(n):
            c = ctypes.c_void_p(None)
            _check(self.lib.sacx_batch_context(self.b, i, ctypes.byref(c)), "sacx_batch_context")
            self.views.append(Solver(self.grids[i], self.params[i], device=dev, stream=self.stream, _borrow=c))
        if init:
            dt = torch.float64
            for i, p in enumerate(problems):
                f = torch.stack([torch.from_numpy(p.fields[k]) for k in FIELDS]).to(dev, dt)
                self.views[i].init_state(f, None, t0=p.t0)

    def __len__(self):
        return self.n

    def __getitem__(self, i) -> Solver:
        return self.views[i]

    def set_tiles(self, threads: int = 0, rows=None):
        arr = None if rows is None else (ctypes.c_int32 * self.n)(*[int(r) for r in rows])
        _check(self.lib.sacx_batch_set_tiles(self.b, int(threads), arr), "sacx_batch_set_tiles")

    def advance(self, nsteps: int, sync: bool = True):
        with torch.cuda.device(self.device):
            _check(self.lib.sacx_batch_advance(self.b, int(nsteps), int(bool(sync))), "sacx_batch_advance")

    def close(self):
        """Destroy the batch (its queued work finishes first)."""
        for v in self.views:
            v.close()
        if self.b:
            with torch.cuda.device(self.device):
                self.lib.sacx_batch_destroy(self.b)
            self.b = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- network calls
class StepGraph:
    """A fixed piece of enqueued work (steps of a context, or of a decomposed
    domain) captured once into a HIP graph through torch.cuda.CUDAGraph and
    replayed: one launch of the graph in place of every kernel launch of the
    piece, for launch-bound runs (small grids, the many small exchange
    kernels of a decomposed domain).  The capture enqueues nothing; each
    replay does the work on the captured stream."""

    def __init__(self, enqueue, stream: torch.cuda.Stream):
        if stream is None or stream.cuda_stream == 0:
            raise ValueError("graph capture needs the work on a stream of its own, not the default stream")
        self.stream = stream
        self.graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph, stream=stream, capture_error_mode="thread_local"):
            enqueue()

    def replay(self):
        with torch.cuda.stream(self.stream):
            self.graph.replay()


def _dp(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(None if t is None else t.data_ptr())


def cnn_buffer_sizes(n: int, h: int, w: int) -> Dict[str, int]:
    lib = load_library()
    s = CnnSizes()
    _check(lib.sacx_cnn_buffer_sizes(int(n), int(h), int(w), ctypes.byref(s)), "sacx_cnn_buffer_sizes")
    return {"input": s.input_bytes, "act": s.act_bytes, "out": s.out_bytes, "work": s.work_bytes}


def cnn_pack(theta: torch.Tensor, packed: torch.Tensor, stream=None):
    lib = load_library()
    st = stream if stream is not None else torch.cuda.current_stream(theta.device)
    with torch.cuda.device(theta.device):
        _check(lib.sacx_cnn_pack(_dp(theta), _dp(packed), ctypes.c_void_p(st.cuda_stream)), "sacx_cnn_pack")


def cnn_forward(packed: torch.Tensor, x: torch.Tensor, act: torch.Tensor, out: torch.Tensor, stream=None):
    """x: (n, h, w, 8) bf16; act: uint8 buffer; out: (n, 10, h, w) float32."""
    lib = load_library()
    n, h, w = x.shape[0], x.shape[1], x.shape[2]
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    with torch.cuda.device(x.device):
        _check(lib.sacx_cnn_forward(_dp(packed), _dp(x), n, h, w, _dp(act), _dp(out), ctypes.c_void_p(st.cuda_stream)),
               "sacx_cnn_forward")


def cnn_backward(packed, x, act, out, target, work, grad, loss, weight=None, stream=None):
    lib = load_library()
    n, h, w = x.shape[0], x.shape[1], x.shape[2]
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    with torch.cuda.device(x.device):
        _check(lib.sacx_cnn_backward(_dp(packed), _dp(x), _dp(act), _dp(out), _dp(target), _dp(weight), n, h, w,
                                     _dp(work),
                                     work.numel() * work.element_size(), _dp(grad), _dp(loss),
                                     ctypes.c_void_p(st.cuda_stream)), "sacx_cnn_backward")


def cnn_backward_noalloc(packed, x, act, out, target, grad, loss, weight=None, stream=None):
    """sacx_cnn_backward on the library's static scratch (no work buffer)."""
    lib = load_library()
    n, h, w = x.shape[0], x.shape[1], x.shape[2]
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    with torch.cuda.device(x.device):
        _check(lib.sacx_cnn_backward_noalloc(_dp(packed), _dp(x), _dp(act), _dp(out), _dp(target), _dp(weight), n, h,
                                             w, _dp(grad), _dp(loss), ctypes.c_void_p(st.cuda_stream)),
               "sacx_cnn_backward_noalloc")


def cnn_adam(theta, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    lib = load_library()
    st = stream if stream is not None else torch.cuda.current_stream(theta.device)
    with torch.cuda.device(theta.device):
        _check(lib.sacx_cnn_adam(_dp(theta), _dp(m), _dp(v), _dp(grad), int(step), float(lr), float(beta1),
                                 float(beta2), float(eps), ctypes.c_void_p(st.cuda_stream)), "sacx_cnn_adam")
