"""Three-dimensional initial states for the 3-D form of the scheme.

Conventions (shared by the 3-D oracle and the GPU library):

* cell-centred grid, x_i = x0 + (i + 1/2) dx, the same in y and z;
* state = eight evolved conserved fields, in this order: rho, m_x, m_y, m_z,
  e (total energy), B_x, B_y, B_z; no background;
* arrays are float64, C-contiguous, shape (nz, ny, nx), x fastest;
* boundaries per side (x-, x+, y-, y+, z-, z+), PERIODIC or OPEN.

Like the 2-D generators this module holds none of the scheme's arithmetic:
only initial data, with e = p/(gamma-1) + rho |v|^2/2 + |B|^2/2.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, Sequence, Tuple

import numpy as np

from .problems import PERIODIC, OPEN, Problem, cell_centres  # noqa: F401

FIELDS3 = ("rho", "mx", "my", "mz", "e", "bx", "by", "bz")


@dataclasses.dataclass
class Problem3:
    name: str
    nx: int
    ny: int
    nz: int
    extent: Tuple[float, float, float, float, float, float]   # x0, x1, y0, y1, z0, z1
    gamma: float
    bc: Tuple[int, int, int, int, int, int]
    fields: Dict[str, np.ndarray]
    t0: float = 0.0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def h(self) -> Tuple[float, float, float]:
        e = self.extent
        return ((e[1] - e[0]) / self.nx, (e[3] - e[2]) / self.ny, (e[5] - e[4]) / self.nz)

    def stacked(self) -> np.ndarray:
        """(8, nz, ny, nx) float64 copy of the evolved fields."""
        return np.stack([self.fields[k] for k in FIELDS3]).astype(np.float64, copy=True)


def conserved3(rho, vx, vy, vz, p, bx, by, bz, gamma, shape) -> Dict[str, np.ndarray]:
    """Conserved fields from primitive ones (each broadcast to `shape`)."""
    b = lambda a: np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))  # noqa: E731
    rho, vx, vy, vz, p, bx, by, bz = (b(a) for a in (rho, vx, vy, vz, p, bx, by, bz))
    e = p / (gamma - 1.0) + 0.5 * rho * ((vx * vx + vy * vy) + vz * vz) + 0.5 * ((bx * bx + by * by) + bz * bz)
    return {"rho": rho, "mx": rho * vx, "my": rho * vy, "mz": rho * vz, "e": e, "bx": bx, "by": by, "bz": bz}


def _grid(nx, ny, nz, extent):
    x = cell_centres(nx, extent[0], extent[1])[None, None, :]
    y = cell_centres(ny, extent[2], extent[3])[None, :, None]
    z = cell_centres(nz, extent[4], extent[5])[:, None, None]
    return x, y, z


def orszag_tang_3d(n: int, ny: int = None, nz: int = None, eps: float = 0.2, b0_scale: float = 1.0) -> Problem3:
    """The Orszag-Tang vortex carried into z on [0, 2pi]^3, periodic, gamma 5/3.

    rho = 25/(36 pi), p = 5/(12 pi), B = B0 (-sin y, sin 2x, 0),
    v = ((1 + eps sin z)(-sin y), (1 + eps sin z) sin x, eps sin z),
    B0 = b0_scale / sqrt(4 pi).  eps = 0 is the 2-D vortex in every z plane;
    eps > 0 makes the flow genuinely three-dimensional (our choice of 3-D
    workload: the paper gives its 3-D results as forthcoming).  div B = 0.
    """
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    ext = (0.0, 2.0 * math.pi) * 3
    x, y, z = _grid(n, ny, nz, ext)
    shape = (nz, ny, n)
    gamma = 5.0 / 3.0
    b0 = b0_scale / math.sqrt(4.0 * math.pi)
    mod = 1.0 + eps * np.sin(z)
    f = conserved3(25.0 / (36.0 * math.pi), -mod * np.sin(y), mod * np.sin(x), eps * np.sin(z) + 0.0 * x,
                   5.0 / (12.0 * math.pi), -b0 * np.sin(y), b0 * np.sin(2.0 * x), 0.0, gamma, shape)
    return Problem3("orszag_tang_3d", n, ny, nz, ext, gamma, (PERIODIC,) * 6, f, meta={"b0": b0, "eps": eps})


def uniform_3d(nx: int, ny: int, nz: int, rho=1.3, v=(0.4, -0.7, 0.25), p=0.9, b=(0.3, 0.8, -0.45),
               gamma=5.0 / 3.0, bc=(PERIODIC,) * 6, extent=(0.0, 1.0, 0.0, 1.0, 0.0, 1.0)) -> Problem3:
    f = conserved3(rho, v[0], v[1], v[2], p, b[0], b[1], b[2], gamma, (nz, ny, nx))
    return Problem3("uniform_3d", nx, ny, nz, tuple(extent), gamma, tuple(bc), f)


def entropy_wave_3d(n: int, amp: float = 0.2, v=(1.0, 0.5, 0.25), p0: float = 1.0, b=(0.3, -0.2, 0.4),
                    gamma: float = 5.0 / 3.0, k=(1, 1, 1)) -> Problem3:
    """rho = 1 + amp sin(2 pi k.x) on [0,1]^3 with uniform v, p and B: an
    exact non-linear solution, the profile advected at v."""
    x, y, z = _grid(n, n, n, (0.0, 1.0) * 3)
    ph = 2.0 * math.pi * ((k[0] * x + k[1] * y) + k[2] * z)
    rho = 1.0 + amp * np.sin(ph)
    f = conserved3(rho, v[0], v[1], v[2], p0, b[0], b[1], b[2], gamma, (n, n, n))
    return Problem3("entropy_wave_3d", n, n, n, (0.0, 1.0) * 3, gamma, (PERIODIC,) * 6, f,
                    meta={"amp": amp, "v": v, "k": k})


def entropy_wave_3d_exact(n: int, t: float, amp: float = 0.2, v=(1.0, 0.5, 0.25), k=(1, 1, 1)) -> np.ndarray:
    """Density of entropy_wave_3d at time t (the initial profile shifted by v t)."""
    x, y, z = _grid(n, n, n, (0.0, 1.0) * 3)
    ph = 2.0 * math.pi * ((k[0] * (x - v[0] * t) + k[1] * (y - v[1] * t)) + k[2] * (z - v[2] * t))
    return np.ascontiguousarray(np.broadcast_to(1.0 + amp * np.sin(ph), (n, n, n)))


def random_smooth_3d(nx: int, ny: int, nz: int, seed: int = 0, amp: float = 0.2, modes: int = 4,
                     gamma: float = 5.0 / 3.0, bc=(PERIODIC,) * 6,
                     extent=(0.0, 1.0, 0.0, 1.0, 0.0, 1.0)) -> Problem3:
    """Positive-density, positive-pressure smooth random state of a few
    Fourier modes (periodic-smooth when the boundaries are periodic)."""
    rng = np.random.default_rng(seed)
    x, y, z = _grid(nx, ny, nz, extent)
    x, y, z = (x - extent[0]) / (extent[1] - extent[0]), (y - extent[2]) / (extent[3] - extent[2]), \
              (z - extent[4]) / (extent[5] - extent[4])

    def field():
        out = np.zeros((nz, ny, nx))
        for _ in range(modes):
            kx, ky, kz = rng.integers(0, 4, size=3)
            ph = rng.uniform(0.0, 2.0 * math.pi)
            a = rng.normal()
            out = out + a * np.cos(2.0 * math.pi * ((kx * x + ky * y) + kz * z) + ph)
        return out / modes

    rho = 1.0 + amp * np.tanh(field())
    p = 1.0 + amp * np.tanh(field())
    vx, vy, vz = 0.5 * field(), 0.5 * field(), 0.5 * field()
    bx, by, bz = 0.5 * field(), 0.5 * field(), 0.5 * field()
    f = conserved3(rho, vx, vy, vz, p, bx, by, bz, gamma, (nz, ny, nx))
    return Problem3("random_smooth_3d", nx, ny, nz, tuple(extent), gamma, tuple(bc), f, meta={"seed": seed})


def embed_2d(prob: Problem, plane: str, depth: int = 1, depth_extent: float = None) -> Problem3:
    """A 2-D problem laid into one plane of a 3-D grid: plane "xy", "xz" or
    "yz" names the 3-D axes of the 2-D x and y; the third axis has `depth`
    cells (periodic; the state does not vary along it) and no velocity or
    field component along it.  Conserved fields are copied exactly."""
    a, b = {"xy": (0, 1), "xz": (0, 2), "yz": (1, 2)}[plane]
    c = 3 - a - b
    n = [0, 0, 0]
    n[a], n[b], n[c] = prob.nx, prob.ny, depth
    ext = [0.0] * 6
    ext[2 * a], ext[2 * a + 1] = prob.x0, prob.x1
    ext[2 * b], ext[2 * b + 1] = prob.y0, prob.y1
    span = prob.dx if depth_extent is None else depth_extent
    ext[2 * c], ext[2 * c + 1] = 0.0, span * depth if depth_extent is None else depth_extent
    bc = [PERIODIC] * 6
    bc[2 * a], bc[2 * a + 1] = prob.bc[0], prob.bc[1]
    bc[2 * b], bc[2 * b + 1] = prob.bc[2], prob.bc[3]

    def lay(arr2):   # (ny2, nx2) -> (nz, ny, nx), 2-D x along axis a, 2-D y along axis b
        out = np.empty((n[2], n[1], n[0]))
        for kk in range(depth):
            if plane == "xy":
                out[kk, :, :] = arr2
            elif plane == "xz":
                out[:, kk, :] = arr2
            else:
                out[:, :, kk] = arr2
        return np.ascontiguousarray(out)

    zero = np.zeros((n[2], n[1], n[0]))
    comp = {0: ("mx", "bx"), 1: ("my", "by"), 2: ("mz", "bz")}
    f = {"rho": lay(prob.fields["rho"]), "e": lay(prob.fields["e"])}
    f[comp[a][0]], f[comp[a][1]] = lay(prob.fields["mx"]), lay(prob.fields["bx"])
    f[comp[b][0]], f[comp[b][1]] = lay(prob.fields["my"]), lay(prob.fields["by"])
    f[comp[c][0]], f[comp[c][1]] = zero.copy(), zero.copy()
    return Problem3(f"{prob.name}_in_{plane}", n[0], n[1], n[2], tuple(ext), prob.gamma, tuple(bc), f,
                    t0=prob.t0, meta={"plane": plane, "depth": depth})


def extract_2d(fields3: np.ndarray, plane: str, index: int = 0) -> np.ndarray:
    """The (6, ny2, nx2) 2-D fields of one plane of an (8, nz, ny, nx) 3-D
    state laid out by embed_2d (2-D order rho, m_x, m_y, e, B_x, B_y)."""
    a, b = {"xy": (0, 1), "xz": (0, 2), "yz": (1, 2)}[plane]
    names = {0: (1, 5), 1: (2, 6), 2: (3, 7)}   # 3-D slots of (m, B) per axis
    if plane == "xy":
        sl = lambda q: fields3[q][index, :, :]   # noqa: E731
    elif plane == "xz":
        sl = lambda q: fields3[q][:, index, :]   # noqa: E731
    else:
        sl = lambda q: fields3[q][:, :, index]   # noqa: E731
    out = [sl(0), sl(names[a][0]), sl(names[b][0]), sl(4), sl(names[a][1]), sl(names[b][1])]
    return np.stack([np.ascontiguousarray(o) for o in out])
