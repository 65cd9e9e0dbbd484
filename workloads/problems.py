"""Initial states for the paper's test problems and for validation problems.

Conventions (shared by the oracle and the GPU library):

* cell-centred grid, x_i = x0 + (i + 1/2) * dx with dx = (x1 - x0) / nx, same in y;
* a 1-D problem has ny = 1, is periodic in y and its y extent equals dx;
* state = six evolved conserved fields, in this order:
  rho~ (density perturbation), m_x, m_y (momentum), e~ (total energy
  perturbation), B~_x, B~_y (field perturbation);
* optional static background: rho_b, e_b, B_bx, B_by (zero when absent);
* arrays are float64, C-contiguous, shape (ny, nx), x fastest;
* boundaries are given per side (x-, x+, y-, y+) as PERIODIC or OPEN.

The total energy density is e = p/(gamma-1) + rho |v|^2 / 2 + |B|^2 / 2
(paper section 2, the closure for the kinetic pressure), which is how
primitive initial data become conserved fields here.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

FIELDS = ("rho", "mx", "my", "e", "bx", "by")
BACKGROUND_FIELDS = ("rho_b", "e_b", "bx_b", "by_b")

PERIODIC = 0
OPEN = 1


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    gamma: float
    bc: Tuple[int, int, int, int]
    fields: Dict[str, np.ndarray]
    background: Optional[Dict[str, np.ndarray]] = None
    t0: float = 0.0
    meta: dict = dataclasses.field(default_factory=dict)
    g: Tuple[float, float] = (0.0, 0.0)   # gravity (x, y)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny

    def copy_fields(self) -> Dict[str, np.ndarray]:
        return {k: np.array(v, dtype=np.float64, copy=True, order="C") for k, v in self.fields.items()}

    def stacked(self) -> np.ndarray:
        """(6, ny, nx) float64 copy of the evolved fields."""
        return np.stack([self.fields[k] for k in FIELDS]).astype(np.float64, copy=True)


def cell_centres(n: int, a: float, b: float) -> np.ndarray:
    d = (b - a) / n
    return a + (np.arange(n, dtype=np.float64) + 0.5) * d


def _conserved(rho, vx, vy, p, bx, by, gamma):
    rho = np.asarray(rho, dtype=np.float64)
    e = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy) + 0.5 * (bx * bx + by * by)
    out = {
        "rho": rho,
        "mx": rho * vx,
        "my": rho * vy,
        "e": e,
        "bx": np.asarray(bx, dtype=np.float64),
        "by": np.asarray(by, dtype=np.float64),
    }
    shape = np.broadcast_shapes(*(np.shape(v) for v in out.values()))
    return {k: np.array(np.broadcast_to(v, shape), dtype=np.float64, order="C", copy=True) for k, v in out.items()}


def orszag_tang(n: int, ny: Optional[int] = None, b0_scale: float = 1.0,
                symmetric: bool = False) -> Problem:
    """Orszag-Tang vortex on [0, 2pi]^2, periodic, gamma = 5/3.

    rho = 25/(36 pi), p = 5/(12 pi), v = (-sin y, sin x),
    B = B0 (-sin y, sin 2x), B0 = b0_scale / sqrt(4 pi).
    The paper's verification section prints a variant on the unit square
    with other wavenumbers; this standard form is the one the workloads use.

    With ``symmetric`` the arrays are made exactly invariant under the
    180-degree rotation (i, j) -> (n-1-i, n-1-j): rho, e even, v, B odd.
    """
    ny = n if ny is None else ny
    gamma = 5.0 / 3.0
    x = cell_centres(n, 0.0, 2.0 * math.pi)[None, :]
    y = cell_centres(ny, 0.0, 2.0 * math.pi)[:, None]
    b0 = b0_scale / math.sqrt(4.0 * math.pi)
    rho = np.full((ny, n), 25.0 / (36.0 * math.pi))
    p = 5.0 / (12.0 * math.pi)
    vx = -np.sin(y) * np.ones_like(x)
    vy = np.sin(x) * np.ones_like(y)
    bx = -b0 * np.sin(y) * np.ones_like(x)
    by = b0 * np.sin(2.0 * x) * np.ones_like(y)
    if symmetric:
        vx, vy, bx, by = (_odd_symmetrise(a) for a in (vx, vy, bx, by))
    f = _conserved(rho, vx, vy, p, bx, by, gamma)
    if symmetric:
        for k in ("rho", "e"):
            f[k] = _even_symmetrise(f[k])
        for k in ("mx", "my"):
            f[k] = _odd_symmetrise(f[k])
    return Problem("orszag_tang", n, ny, 0.0, 2.0 * math.pi, 0.0, 2.0 * math.pi, gamma,
                   (PERIODIC,) * 4, f, meta={"b0": b0})


def _rot180(a):
    return a[::-1, ::-1]


def _odd_symmetrise(a):
    a = np.array(a, dtype=np.float64)
    ny, nx = a.shape
    # keep the lower half (in flattened order), mirror it with a sign flip
    flat = a.reshape(-1)
    n = flat.size
    out = flat.copy()
    half = n // 2
    out[n - half:] = -flat[:half][::-1]
    if n % 2 == 1:
        out[half] = 0.0
    return out.reshape(ny, nx)


def _even_symmetrise(a):
    a = np.array(a, dtype=np.float64)
    ny, nx = a.shape
    flat = a.reshape(-1)
    n = flat.size
    out = flat.copy()
    half = n // 2
    out[n - half:] = flat[:half][::-1]
    return out.reshape(ny, nx)


def brio_wu(n: int = 800, s_left: float = 1.0, s_right: float = 1.0,
            along_y: bool = False) -> Problem:
    """Brio-Wu shock tube on [0, 1], gamma = 2, open ends.

    Left  (x_i < 0.5): rho = 1,     p = 1,   v = 0, B = (0.75,  1)
    Right (x_i >= 0.5): rho = 0.125, p = 0.1, v = 0, B = (0.75, -1)
    ``s_left``/``s_right`` scale rho and p of one side (batched instances);
    B_x is never scaled, so div B stays zero.
    With ``along_y`` the tube lies along y in a 1 x n grid, components swapped.
    """
    gamma = 2.0
    xc = cell_centres(n, 0.0, 1.0)
    left = xc < 0.5
    rho = np.where(left, 1.0 * s_left, 0.125 * s_right)
    p = np.where(left, 1.0 * s_left, 0.1 * s_right)
    bn = np.full(n, 0.75)
    bt = np.where(left, 1.0, -1.0)
    z = np.zeros(n)
    dx = 1.0 / n
    if not along_y:
        f = _conserved(rho[None, :], z[None, :], z[None, :], p[None, :], bn[None, :], bt[None, :], gamma)
        return Problem("brio_wu", n, 1, 0.0, 1.0, 0.0, dx, gamma, (OPEN, OPEN, PERIODIC, PERIODIC), f,
                       meta={"s_left": s_left, "s_right": s_right})
    f = _conserved(rho[:, None], z[:, None], z[:, None], p[:, None], bt[:, None], bn[:, None], gamma)
    return Problem("brio_wu_y", 1, n, 0.0, dx, 0.0, 1.0, gamma, (PERIODIC, PERIODIC, OPEN, OPEN), f,
                   meta={"s_left": s_left, "s_right": s_right})


def uniform_state(nx: int, ny: int, rho=1.3, v=(0.4, -0.7), p=0.9, b=(0.3, 0.8),
                  gamma=5.0 / 3.0, bc=(PERIODIC,) * 4, extent=(1.0, 1.0)) -> Problem:
    f = _conserved(np.full((ny, nx), rho), np.full((ny, nx), v[0]), np.full((ny, nx), v[1]),
                   np.full((ny, nx), p), np.full((ny, nx), b[0]), np.full((ny, nx), b[1]), gamma)
    return Problem("uniform", nx, ny, 0.0, extent[0], 0.0, extent[1], gamma, tuple(bc), f)


def entropy_wave(n: int, amp: float = 0.2, rho0: float = 1.0, v0: float = 1.0,
                 p0: float = 1.0, b=(0.0, 0.0), gamma: float = 5.0 / 3.0, k: int = 1) -> Problem:
    """rho = rho0 (1 + amp sin(2 pi k x)) on [0,1], uniform v = (v0, 0), p, B.

    An exact non-linear solution of ideal MHD: the density profile is
    advected at v0 with nothing else changing.
    """
    x = cell_centres(n, 0.0, 1.0)[None, :]
    rho = rho0 * (1.0 + amp * np.sin(2.0 * math.pi * k * x))
    one = np.ones_like(rho)
    f = _conserved(rho, v0 * one, 0.0 * one, p0 * one, b[0] * one, b[1] * one, gamma)
    return Problem("entropy_wave", n, 1, 0.0, 1.0, 0.0, 1.0 / n, gamma, (PERIODIC,) * 4, f,
                   meta={"amp": amp, "rho0": rho0, "v0": v0, "p0": p0, "k": k})


def sound_wave(n: int, eps: float = 1e-8, rho0: float = 1.0, p0: float = 0.6,
               gamma: float = 5.0 / 3.0, bx: float = 0.0, k: int = 1) -> Problem:
    """Right-moving linear sound wave along x on [0, 1] (B parallel to k or zero).

    delta rho = eps rho0 cos(kx), delta v_x = eps c_s cos(kx),
    delta p = eps gamma p0 cos(kx), with c_s = sqrt(gamma p0 / rho0).
    """
    x = cell_centres(n, 0.0, 1.0)[None, :]
    cs = math.sqrt(gamma * p0 / rho0)
    c = np.cos(2.0 * math.pi * k * x)
    rho = rho0 * (1.0 + eps * c)
    vx = eps * cs * c
    p = p0 * (1.0 + gamma * eps * c)
    one = np.ones_like(rho)
    f = _conserved(rho, vx, 0.0 * one, p, bx * one, 0.0 * one, gamma)
    return Problem("sound_wave", n, 1, 0.0, 1.0, 0.0, 1.0 / n, gamma, (PERIODIC,) * 4, f,
                   meta={"eps": eps, "rho0": rho0, "p0": p0, "cs": cs, "k": k})


def alfven_wave(n: int, eps: float = 1e-8, rho0: float = 1.0, p0: float = 0.6,
                b0: float = 0.8, gamma: float = 5.0 / 3.0, k: int = 1) -> Problem:
    """Right-moving linear Alfven wave along x on [0, 1].

    B = (b0, -eps b0 cos kx), v_y = eps v_A cos kx, v_A = b0 / sqrt(rho0).
    """
    x = cell_centres(n, 0.0, 1.0)[None, :]
    va = b0 / math.sqrt(rho0)
    c = np.cos(2.0 * math.pi * k * x)
    one = np.ones_like(c)
    f = _conserved(rho0 * one, 0.0 * one, eps * va * c, p0 * one, b0 * one, -eps * b0 * c, gamma)
    return Problem("alfven_wave", n, 1, 0.0, 1.0, 0.0, 1.0 / n, gamma, (PERIODIC,) * 4, f,
                   meta={"eps": eps, "rho0": rho0, "p0": p0, "b0": b0, "va": va, "k": k})


def random_smooth(nx: int, ny: int, seed: int = 0, amp: float = 0.2, modes: int = 4,
                  gamma: float = 5.0 / 3.0, bc=(PERIODIC,) * 4,
                  extent=(1.0, 1.0)) -> Problem:
    """Positive-density, positive-pressure smooth random state (a few Fourier modes).

    Not periodic-smooth unless bc is periodic; for OPEN boundaries it is just
    a generic smooth state.
    """
    rng = np.random.default_rng(seed)
    x = cell_centres(nx, 0.0, extent[0])[None, :] / extent[0]
    y = cell_centres(ny, 0.0, extent[1])[:, None] / extent[1]

    def field():
        out = np.zeros((ny, nx))
        for _ in range(modes):
            kx, ky = rng.integers(0, 4, size=2)
            ph = rng.uniform(0.0, 2.0 * math.pi)
            a = rng.normal()
            out = out + a * np.cos(2.0 * math.pi * (kx * x + ky * y) + ph)
        return out / modes

    rho = 1.0 + amp * np.tanh(field())
    p = 1.0 + amp * np.tanh(field())
    vx, vy = 0.5 * field(), 0.5 * field()
    bx, by = 0.5 * field(), 0.5 * field()
    f = _conserved(rho, vx, vy, p, bx, by, gamma)
    return Problem("random_smooth", nx, ny, 0.0, extent[0], 0.0, extent[1], gamma, tuple(bc), f,
                   meta={"seed": seed})


def split_background(prob: Problem, rho_b: float, e_b: float, b_b=(0.0, 0.0)) -> Problem:
    """Move uniform parts into the static background: rho = rho_b + rho~ etc.

    The background is uniform, hence in (magneto)hydrostatic equilibrium with
    no gravity; the split and unsplit runs describe the same state.
    """
    shape = (prob.ny, prob.nx)
    bg = {
        "rho_b": np.full(shape, rho_b),
        "e_b": np.full(shape, e_b),
        "bx_b": np.full(shape, b_b[0]),
        "by_b": np.full(shape, b_b[1]),
    }
    f = prob.copy_fields()
    f["rho"] = f["rho"] - rho_b
    f["e"] = f["e"] - e_b
    f["bx"] = f["bx"] - b_b[0]
    f["by"] = f["by"] - b_b[1]
    return dataclasses.replace(prob, name=prob.name + "_split", fields=f, background=bg)


def with_gravity(prob: Problem, g: Tuple[float, float]) -> Problem:
    """The same initial state under a uniform gravity g = (g_x, g_y)."""
    return dataclasses.replace(prob, name=prob.name + "_g", g=(float(g[0]), float(g[1])))


def stratified_atmosphere(nx: int, ny: int, g0: float = 1.0, scale_height: float = 0.25, rho0: float = 1.0,
                          b_b=(0.0, 0.0), amp: float = 0.02, width: float = 0.05, centre=(0.5, 0.15),
                          gamma: float = 5.0 / 3.0, extent=(1.0, 1.0)) -> Problem:
    """A gravitationally stratified atmosphere carrying a wave pulse, the
    kind of medium the code exists for (section 1: waves in a strongly
    magnetised, stratified solar atmosphere).

    Background (static, in equilibrium): isothermal under g = (0, -g0) with
    scale height H, rho_b = rho0 exp(-y/H) and p_b = rho_b g0 H, so that
    dp_b/dy = -rho_b g0; a uniform field B_b (force-free);
    e_b = p_b/(gamma-1) + |B_b|^2/2.  Perturbation: a Gaussian vertical
    velocity pulse of peak `amp` times the sound speed, m~ = rho_b v,
    e~ = rho_b v^2/2 (no pressure perturbation), rho~ = B~ = 0.
    x periodic, y open (zero-gradient), domain [0, Lx] x [0, Ly].
    """
    lx, ly = extent
    x = cell_centres(nx, 0.0, lx)
    y = cell_centres(ny, 0.0, ly)
    X, Y = np.meshgrid(x, y)
    H = scale_height
    rho_b = rho0 * np.exp(-Y / H)
    p_b = rho_b * g0 * H
    cs = math.sqrt(gamma * g0 * H)
    r2 = ((X - centre[0] * lx) ** 2 + (Y - centre[1] * ly) ** 2) / width ** 2
    vy = amp * cs * np.exp(-r2)
    zero = np.zeros_like(X)
    b2 = b_b[0] ** 2 + b_b[1] ** 2
    fields = {"rho": zero.copy(), "mx": zero.copy(), "my": rho_b * vy, "e": 0.5 * rho_b * vy * vy,
              "bx": zero.copy(), "by": zero.copy()}
    bg = {"rho_b": rho_b, "e_b": p_b / (gamma - 1.0) + 0.5 * b2, "bx_b": np.full_like(X, b_b[0]),
          "by_b": np.full_like(X, b_b[1])}
    return Problem(f"stratified_{nx}x{ny}", nx, ny, 0.0, lx, 0.0, ly, gamma, (PERIODIC, PERIODIC, OPEN, OPEN),
                   fields, bg, 0.0, {"g0": g0, "H": H, "amp": amp}, (0.0, -g0))


def transpose_problem(prob: Problem) -> Problem:
    """Same problem with x and y exchanged (fields transposed, components swapped)."""
    f = prob.fields
    g = {
        "rho": f["rho"].T.copy(),
        "mx": f["my"].T.copy(),
        "my": f["mx"].T.copy(),
        "e": f["e"].T.copy(),
        "bx": f["by"].T.copy(),
        "by": f["bx"].T.copy(),
    }
    bc = (prob.bc[2], prob.bc[3], prob.bc[0], prob.bc[1])
    bg = None
    if prob.background is not None:
        b = prob.background
        bg = {"rho_b": b["rho_b"].T.copy(), "e_b": b["e_b"].T.copy(),
              "bx_b": b["by_b"].T.copy(), "by_b": b["bx_b"].T.copy()}
    return Problem(prob.name + "_T", prob.ny, prob.nx, prob.y0, prob.y1, prob.x0, prob.x1,
                   prob.gamma, bc, g, bg, prob.t0, dict(prob.meta), (prob.g[1], prob.g[0]))


def batch_instances(seed: int = 0, n_bw: int = 32, n_ot: int = 32) -> List[Problem]:
    """The mixed batch: Brio-Wu tubes then Orszag-Tang boxes, seeded draws.

    Draw order: for each tube (N in [400, 3200], s_L, s_R in U(0.5, 2)),
    then for each box (side in [128, 768], B0 factor in U(0.5, 1.5)).
    """
    rng = np.random.default_rng(seed)
    out: List[Problem] = []
    for _ in range(n_bw):
        n = int(rng.integers(400, 3201))
        sl = float(rng.uniform(0.5, 2.0))
        sr = float(rng.uniform(0.5, 2.0))
        out.append(brio_wu(n, sl, sr))
    for _ in range(n_ot):
        side = int(rng.integers(128, 769))
        b = float(rng.uniform(0.5, 1.5))
        out.append(orszag_tang(side, b0_scale=b))
    return out


def synthetic_ratio_planes(nx: int, ny: int, seed: int = 0, tile: int = 8, frac_plain: float = 0.25) -> np.ndarray:
    """Seeded coefficient-ratio planes (10, ny, nx) float32 for the supplied-ratio
    path: values uniform in [0, 4], with a random fraction of tile x tile blocks
    (all 10 planes) set to -1, which asks for the plain ratio there."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.0, 4.0, size=(10, ny, nx)).astype(np.float32)
    for ty in range(-(-ny // tile)):
        for tx in range(-(-nx // tile)):
            if rng.uniform() < frac_plain:
                r[:, ty * tile:(ty + 1) * tile, tx * tile:(tx + 1) * tile] = -1.0
    return r


def cnn_case(n: int, h: int, w: int, seed: int = 0):
    """Seeded network test case: parameters (He-scaled, small random biases),
    input images (n, 6, h, w) and target ratio planes (n, 10, h, w) in [0, 4]."""
    rng = np.random.default_rng(seed)
    layers = [(6, 32), (32, 32), (32, 32), (32, 10)]
    p = {}
    for l, (ci, co) in enumerate(layers):
        p[f"w{l}"] = rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), size=(co, ci, 3, 3))
        p[f"b{l}"] = rng.normal(0.0, 0.1, size=co)
    x = rng.normal(0.0, 1.0, size=(n, 6, h, w))
    t = rng.uniform(0.0, 4.0, size=(n, 10, h, w))
    return p, x, t
