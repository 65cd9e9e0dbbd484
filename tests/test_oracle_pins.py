"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test would fail on a plausible mistake somewhere in the oracle: a wrong
stencil coefficient, a dropped flux term, a wrong sign or index, a transposed
operand, a wrong Runge-Kutta weight, a wrong hyper-diffusion window.
"""

import itertools
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pressure(f, gamma, bg=None):
    rho = f["rho"] + (bg["rho_b"] if bg else 0.0)
    e = f["e"] + (bg["e_b"] if bg else 0.0)
    bx = f["bx"] + (bg["bx_b"] if bg else 0.0)
    by = f["by"] + (bg["by_b"] if bg else 0.0)
    return (gamma - 1.0) * (e - 0.5 * (f["mx"] ** 2 + f["my"] ** 2) / rho - 0.5 * (bx ** 2 + by ** 2))


# ---------------------------------------------------------------- D operator

def test_deriv_exact_on_quartics(oracle_lib):
    """Fourth-order central difference (section 2) is exact for degree <= 4."""
    n, h = 48, 0.05
    x = (np.arange(n) - n / 2) * h
    rng = np.random.default_rng(1)
    for deg in range(5):
        a = rng.normal(size=deg + 1)
        f = sum(a[k] * x ** k for k in range(deg + 1))
        df = sum(k * a[k] * x ** (k - 1) for k in range(1, deg + 1)) if deg else 0 * x
        d = oracle_lib.deriv_line(f, h)
        inner = slice(2, n - 2)  # away from the periodic wrap
        assert np.max(np.abs(d[inner] - df[inner])) < 1e-12


def test_deriv_quintic_truncation_error(oracle_lib):
    """D x^5 = 5 x^4 - 4 h^4: the leading error term -h^4 f^(5) / 30."""
    n, h = 48, 0.05
    x = (np.arange(n) - n / 2) * h
    d = oracle_lib.deriv_line(x ** 5, h)
    inner = slice(2, n - 2)
    assert np.max(np.abs(d[inner] - (5 * x[inner] ** 4 - 4 * h ** 4))) < 1e-12


def test_deriv_fourier_symbol(oracle_lib):
    """On e^{ikx} the operator multiplies by i (8 sin kh - sin 2kh) / (6h)."""
    n = 64
    h = 1.0 / n
    x = np.arange(n) * h
    for k in (1, 3, 7, 16, 25, 31):
        th = 2 * math.pi * k * h
        d = oracle_lib.deriv_line(np.sin(2 * math.pi * k * x), h)
        expect = (8 * math.sin(th) - math.sin(2 * th)) / (6 * h) * np.cos(2 * math.pi * k * x)
        assert np.max(np.abs(d - expect)) <= 1e-12 * max(1.0, np.max(np.abs(expect)))


# ------------------------------------------------------- hyper-diffusion ratio

def _golden_rows():
    rows = []
    with open(os.path.join(GOLDEN, "hd_ratio_hand.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, q, faces, expect = [p.strip() for p in line.split("|")]
            rows.append((name, np.array([float(v) for v in q.split()]),
                         [int(v) for v in faces.split()], [float(v) for v in expect.split()]))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: r[0])
def test_hd_ratio_hand_computed(oracle_lib, row):
    name, q, faces, expect = row
    R = oracle_lib.hd_ratio_line(q)
    got = [R[i] for i in faces]
    assert got == expect, (name, got, expect)


def test_hd_ratio_bound_exhaustive(oracle_lib):
    """0 <= R <= 4 on every binary line of length 12 (brute force), and the
    bound is reached (by the checkerboard)."""
    worst = 0.0
    for bits in itertools.product((0.0, 1.0), repeat=12):
        R = oracle_lib.hd_ratio_line(np.array(bits))
        assert np.all(R >= 0.0)
        worst = max(worst, float(R.max()))
    assert worst == 4.0


def test_hd_ratio_properties(oracle_lib):
    rng = np.random.default_rng(7)
    for trial in range(200):
        n = int(rng.integers(8, 40))
        q = rng.normal(size=n) * rng.choice([1e-6, 1.0, 1e6])
        R = oracle_lib.hd_ratio_line(q)
        assert np.all(R >= 0.0) and np.all(R <= 4.0 * (1 + 1e-15))
        # invariant under scaling by a power of two (exact) and nearly under shifts
        assert np.array_equal(oracle_lib.hd_ratio_line(q * 8.0), R)
        R2 = oracle_lib.hd_ratio_line(q * 3.0 + 0.25 * np.max(np.abs(q)))
        assert np.allclose(R2, R, rtol=1e-9, atol=1e-9)
        # mirror image: face i+1/2 of the reversed line is face n-2-i of the original
        Rm = oracle_lib.hd_ratio_line(q[::-1].copy())
        assert np.array_equal(Rm[: n - 1], R[: n - 1][::-1])


# ----------------------------------------------------------- whole scheme

def test_uniform_states_bitwise(oracle_lib):
    """Every difference of a uniform state is exactly 0 (and R = 0), so a
    uniform state must not change by a single bit, with any boundaries,
    background or hyper-diffusion."""
    cases = [
        W.uniform_state(20, 12),
        W.uniform_state(17, 9, bc=(W.problems.OPEN,) * 4),
        W.uniform_state(30, 1, bc=(W.problems.OPEN, W.problems.OPEN, 0, 0), extent=(1.0, 1.0 / 30)),
        W.split_background(W.uniform_state(16, 16), 0.4, 0.5, (0.1, -0.2)),
    ]
    for prob in cases:
        s = oracle_lib.State(prob)
        s.run(40)
        for k, v in prob.fields.items():
            assert np.array_equal(s.fields()[k], v), (prob.name, k)


def _entropy_err(oracle_lib, n, t_end=0.5, amp=0.2):
    prob = W.entropy_wave(n, amp=amp)
    s = oracle_lib.State(prob, hd_on=False)
    s.run(100000, t_end=t_end)
    assert abs(s.t - t_end) <= 1e-12 * t_end
    x = W.cell_centres(n, 0.0, 1.0)
    exact = 1.0 * (1.0 + amp * np.sin(2 * math.pi * (x - 1.0 * s.t)))
    return float(np.sqrt(np.mean((s.fields()["rho"][0] - exact) ** 2)))


def test_entropy_wave_fourth_order(oracle_lib):
    """The advected density profile is an exact solution; fourth-order space
    and time discretisation give error ~ N^-4 (section 2)."""
    ns = [16, 32, 64, 128]
    errs = [_entropy_err(oracle_lib, n) for n in ns]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert orders[-1] >= 3.9 and orders[-2] >= 3.8, (errs, orders)


def _propagate(f0_hat, k_idx, n, h, speed, dts):
    """Apply the RK4 amplification of d/dt u = -speed D u mode by mode."""
    th = 2 * math.pi * k_idx / n
    ktil = (8 * np.sin(th) - np.sin(2 * th)) / (6 * h)
    out = f0_hat.astype(complex)
    for dt in dts:
        z = -1j * speed * ktil * dt
        g = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        out = out * g
    return out


def _run_recording_dt(oracle_lib, prob, nsteps, **kw):
    s = oracle_lib.State(prob, **kw)
    dts = []
    for _ in range(nsteps):
        s.run(1)
        dts.append(float(s.last[0]))
    return s, dts


def test_entropy_wave_discrete_propagator(oracle_lib):
    """At any amplitude m = v0 rho is kept by every stage, so rho follows the
    linear semi-discrete system d rho/dt = -v0 D rho exactly: compare with the
    FFT discrete propagator (modified wavenumber x RK4 amplification)."""
    n = 32
    prob = W.entropy_wave(n, amp=0.3, v0=0.7, k=2)
    s, dts = _run_recording_dt(oracle_lib, prob, 60, hd_on=False)
    rho0 = prob.fields["rho"][0]
    kk = np.fft.fftfreq(n, d=1.0 / n)
    expect = np.real(np.fft.ifft(_propagate(np.fft.fft(rho0), kk, n, 1.0 / n, 0.7, dts)))
    got = s.fields()["rho"][0]
    assert np.linalg.norm(got - expect) / np.linalg.norm(expect) < 1e-12


@pytest.mark.parametrize("kind", ["sound", "alfven"])
def test_linear_waves(oracle_lib, kind):
    """Small-amplitude sound and Alfven waves: against the FFT discrete
    propagator (tight) and against the closed form omega = c k (O(k^4 h^4))."""
    n, eps = 64, 1e-8
    if kind == "sound":
        prob = W.sound_wave(n, eps=eps)
        speed = prob.meta["cs"]
        pick = lambda f: (f["rho"][0] - 1.0) / eps           # noqa: E731
        amp0 = 1.0
    else:
        prob = W.alfven_wave(n, eps=eps)
        speed = prob.meta["va"]
        pick = lambda f: (f["my"][0] / f["rho"][0]) / eps    # noqa: E731
        amp0 = prob.meta["va"]
    s, dts = _run_recording_dt(oracle_lib, prob, 120, hd_on=False)
    got = pick(s.fields())
    x = W.cell_centres(n, 0.0, 1.0)
    u0 = amp0 * np.cos(2 * math.pi * x)
    kk = np.fft.fftfreq(n, d=1.0 / n)
    disc = np.real(np.fft.ifft(_propagate(np.fft.fft(u0), kk, n, 1.0 / n, speed, dts)))
    assert np.linalg.norm(got - disc) / np.linalg.norm(disc) < 1e-6
    t = sum(dts)
    exact = amp0 * np.cos(2 * math.pi * (x - speed * t))
    kh = 2 * math.pi / n
    bound = 3 * (2 * math.pi) * speed * t * kh ** 4 / 30 + 1e-6
    assert np.max(np.abs(got - exact)) / amp0 < bound


@pytest.mark.parametrize("hd_on", [False, True])
def test_conservation_periodic(oracle_lib, hd_on):
    """Every term is in flux form, so with periodic boundaries the sums of
    rho~, m, e~, B~ do not change."""
    for prob in (W.orszag_tang(40), W.random_smooth(36, 28, seed=3)):
        s = oracle_lib.State(prob, hd_on=hd_on)
        before = s.sums()
        scale = oracle_lib.sums(s.cfg, [np.abs(a) for a in s.f])
        s.run(40)
        after = s.sums()
        assert np.all(np.abs(after - before) <= 1e-13 * np.maximum(scale, 1e-300)), (after - before) / scale


def _div_b(f, dx, dy):
    def d(a, ax, h):
        return (8 * (np.roll(a, -1, ax) - np.roll(a, 1, ax)) - (np.roll(a, -2, ax) - np.roll(a, 2, ax))) / (12 * h)
    return d(f["bx"], 1, dx) + d(f["by"], 0, dy)


def test_div_b_preserved_without_hd(oracle_lib):
    """Central differences keep the discrete div B (section 2); OT starts at 0."""
    prob = W.orszag_tang(48)
    s = oracle_lib.State(prob, hd_on=False)
    s.run(60)
    f = s.fields()
    bmax = max(np.max(np.abs(f["bx"])), np.max(np.abs(f["by"])))
    assert np.max(np.abs(_div_b(f, prob.dx, prob.dy))) <= 1e-12 * bmax / prob.dx


def test_brio_wu_bx_constant_bitwise(oracle_lib):
    """In 1-D the normal field has no flux of any kind: B_x stays 0.75 exactly."""
    s = oracle_lib.State(W.brio_wu(800))
    s.run(100000, t_end=0.02)
    assert np.all(s.fields()["bx"] == 0.75)


def test_brio_wu_fast_fronts_and_positivity(oracle_lib):
    """Brio-Wu to t = 0.1 (section 5.2 states; gamma = 2): rho, p stay positive,
    the outer states are untouched ahead of the fast rarefactions, and the
    fronts have reached x = 0.5 -+ 0.9 c_f t, with c_f = sqrt((gamma p + B^2)/rho)
    of each side."""
    prob = W.brio_wu(800)
    s = oracle_lib.State(prob)
    s.run(100000, t_end=0.1)
    f = s.fields()
    p = pressure(f, 2.0)[0]
    rho = f["rho"][0]
    assert rho.min() > 0 and p.min() > 0
    x = W.cell_centres(800, 0.0, 1.0)
    cl = math.sqrt((2 * 1.0 + 0.75 ** 2 + 1.0) / 1.0)
    cr = math.sqrt((2 * 0.1 + 0.75 ** 2 + 1.0) / 0.125)
    t = s.t
    far_l = x < 0.5 - 1.1 * cl * t
    far_r = x > 0.5 + 1.1 * cr * t
    assert np.max(np.abs(rho[far_l] - 1.0)) < 1e-4 and np.max(np.abs(rho[far_r] - 0.125)) < 1e-4
    i_l = np.argmin(np.abs(x - (0.5 - 0.9 * cl * t)))
    i_r = np.argmin(np.abs(x - (0.5 + 0.9 * cr * t)))
    assert abs(rho[i_l] - 1.0) > 1e-3 and abs(rho[i_r] - 0.125) > 1e-4
    # extrema bounded by the initial data (small overshoot allowed)
    assert rho.max() < 1.0 + 1e-4 and rho.min() > 0.9 * 0.125


def test_hd_needed_for_brio_wu(oracle_lib):
    """Without hyper-diffusion the central scheme breaks down at the shock
    (section 2: the central scheme alone is unstable for shocks)."""
    s = oracle_lib.State(W.brio_wu(800), hd_on=False)
    rc, done = s.advance(200, t_end=0.1)
    assert rc == oracle_lib.ENONPHYS and done < 200


def test_orszag_tang_point_symmetry_bitwise(oracle_lib):
    """The OT vortex is symmetric under the 180-degree rotation; with a
    symmetric initial state every operation is mirror-exact."""
    prob = W.orszag_tang(40, symmetric=True)
    s = oracle_lib.State(prob)
    s.run(60)
    f = s.fields()
    r = lambda a: a[::-1, ::-1]   # noqa: E731
    for k in ("rho", "e"):
        assert np.array_equal(f[k], r(f[k])), k
    for k in ("mx", "my", "bx", "by"):
        assert np.array_equal(f[k], -r(f[k])), k


def test_transpose_brio_wu_bitwise(oracle_lib):
    """The y code path: the tube along y equals the tube along x."""
    a = oracle_lib.State(W.brio_wu(400))
    b = oracle_lib.State(W.brio_wu(400, along_y=True))
    a.run(100000, t_end=0.05)
    b.run(100000, t_end=0.05)
    assert a.steps == b.steps and a.t == b.t
    fa, fb = a.fields(), b.fields()
    for ka, kb in (("rho", "rho"), ("mx", "my"), ("my", "mx"), ("e", "e"), ("bx", "by"), ("by", "bx")):
        assert np.array_equal(fa[ka][0], fb[kb][:, 0]), ka


def test_transpose_2d_bitwise(oracle_lib):
    """2-D with cross terms: x <-> y exchange commutes with the scheme."""
    p = W.random_smooth(24, 18, seed=11)
    q = W.transpose_problem(p)
    a, b = oracle_lib.State(p), oracle_lib.State(q)
    a.run(15)
    b.run(15)
    fa, fb = a.fields(), b.fields()
    for ka, kb in (("rho", "rho"), ("mx", "my"), ("my", "mx"), ("e", "e"), ("bx", "by"), ("by", "bx")):
        assert np.array_equal(fa[ka], fb[kb].T), ka


def test_mirror_x_rhs_bitwise(oracle_lib):
    """x -> -x: rho, m_y, e, B_y even; m_x, B_x odd; the right-hand side too."""
    p = W.random_smooth(26, 20, seed=5)
    f = p.fields
    m = {k: (-1 if k in ("mx", "bx") else 1) * f[k][:, ::-1].copy() for k in f}
    pm = W.Problem("mirror", p.nx, p.ny, p.x0, p.x1, p.y0, p.y1, p.gamma, p.bc, m)
    a, b = oracle_lib.State(p), oracle_lib.State(pm)
    Ka, Kb = a.rhs(1.7), b.rhs(1.7)
    for i, k in enumerate(W.FIELDS):
        sgn = -1 if k in ("mx", "bx") else 1
        assert np.array_equal(Kb[i], sgn * Ka[i][:, ::-1]), k


def test_split_equals_unsplit(oracle_lib):
    """Moving a uniform part into the static background (SAC split form)
    describes the same physics: totals agree after 40 steps."""
    prob = W.orszag_tang(40)
    gamma = prob.gamma
    rho0, p0 = 25 / (36 * math.pi), 5 / (12 * math.pi)
    bb = (0.05, -0.08)
    sp = W.split_background(prob, rho0 / 2, p0 / (2 * (gamma - 1)) + 0.5 * (bb[0] ** 2 + bb[1] ** 2), bb)
    a, b = oracle_lib.State(prob), oracle_lib.State(sp)
    a.run(40)
    b.run(40)
    fa, fb = a.fields(), b.fields()
    tot = {"rho": "rho_b", "e": "e_b", "bx": "bx_b", "by": "by_b"}
    for k in W.FIELDS:
        v = fb[k] + (sp.background[tot[k]] if k in tot else 0.0)
        assert oracle_lib.rel_l2(v, fa[k]) < 1e-12, k


def test_resume_bitwise(oracle_lib):
    prob = W.orszag_tang(32)
    a = oracle_lib.State(prob)
    a.run(30)
    b = oracle_lib.State(prob)
    b.run(12)
    b.run(18)
    assert a.t == b.t
    assert np.array_equal(a.stacked(), b.stacked())


def test_non_physical_state_detected(oracle_lib):
    prob = W.orszag_tang(24)
    prob.fields["e"][5, 7] = 0.0   # kinetic + magnetic energy exceed e: p < 0
    s = oracle_lib.State(prob)
    rc, done = s.advance(5)
    assert rc == oracle_lib.ENONPHYS and done == 0
    assert np.array_equal(s.fields()["e"], prob.fields["e"])


def test_cfl_dt_closed_form(oracle_lib):
    """dt = CFL min_d h_d / (|v_d| + c_f) with c_f = sqrt((gamma p + |B|^2) / rho)."""
    prob = W.uniform_state(10, 8, rho=1.3, v=(0.4, -0.7), p=0.9, b=(0.3, 0.8), extent=(1.0, 0.5))
    cx, cy, cmax, dt = oracle_lib.State(prob, cfl=0.3).wavespeed()
    cf = math.sqrt((5 / 3 * 0.9 + 0.3 ** 2 + 0.8 ** 2) / 1.3)
    assert math.isclose(cx, 0.4 + cf, rel_tol=1e-14) and math.isclose(cy, 0.7 + cf, rel_tol=1e-14)
    assert math.isclose(cmax, 0.7 + cf, rel_tol=1e-14)
    assert math.isclose(dt, 0.3 * min(0.1 / (0.4 + cf), 0.0625 / (0.7 + cf)), rel_tol=1e-14)


def test_hd_damps_grid_scale_noise(oracle_lib):
    """A grid-scale (checkerboard) density ripple on a uniform state is not
    seen by the central operator (its symbol vanishes at k h = pi) but is
    removed by the hyper-diffusion (R = 4 there)."""
    prob = W.uniform_state(32, 1, v=(0.0, 0.0), b=(0.0, 0.0), extent=(1.0, 1.0 / 32))
    ripple = 1e-3 * (-1.0) ** np.arange(32)
    prob.fields["rho"] = prob.fields["rho"] + ripple[None, :]
    prob.fields["e"] = prob.fields["e"].copy()
    amp = lambda s: np.abs(np.sum((s.fields()["rho"][0] - 1.3) * (-1.0) ** np.arange(32))) / 32  # noqa: E731
    on, off = oracle_lib.State(prob), oracle_lib.State(prob, hd_on=False)
    on.run(50)
    off.run(50)
    assert amp(off) > 0.9e-3 and amp(on) < 0.5 * amp(off)


def test_patch_step_matches_full_step(oracle_lib):
    """The patch entry point (used for sampled checks of large GPU runs) gives
    exactly the full-domain step on the patch interior."""
    prob = W.orszag_tang(48)
    s = oracle_lib.State(prob)
    cx, cy, cmax, dt = s.wavespeed()
    f0 = s.stacked()
    s.run(1)
    assert s.last[0] == dt and s.last[1] == cmax
    full = s.stacked()
    i0, j0, w, h = 30, 5, 40, 33   # wraps around the right edge
    ii = (np.arange(i0, i0 + w) % 48)
    jj = (np.arange(j0, j0 + h) % 48)
    patch = [f0[k][np.ix_(jj, ii)] for k in range(6)]
    out = oracle_lib.step_patch(s.cfg, patch, None, dt, cmax)
    ref = np.stack([full[k][np.ix_(jj[12:-12], ii[12:-12])] for k in range(6)])
    assert np.array_equal(out, ref)


# ------------------------------------------- hyper-diffusion: physical pins

def _hd_only(oracle_lib, prob, cmax, **kw):
    on = oracle_lib.State(prob, **kw).rhs(cmax)
    off = oracle_lib.State(prob, hd_on=False).rhs(cmax)
    return on - off


def _prims(prob):
    f = prob.fields
    rho = f["rho"]
    return rho, f["mx"] / rho, f["my"] / rho, f["bx"], f["by"]


def _heating(prob, K):
    """Rate of change of the thermal energy e - rho v^2/2 - B^2/2 implied by K."""
    rho, vx, vy, bx, by = _prims(prob)
    return (K[3] - (vx * K[1] + vy * K[2]) + 0.5 * (vx * vx + vy * vy) * K[0]
            - (bx * K[4] + by * K[5]))


@pytest.mark.parametrize("kind", ["viscous", "ohmic"])
def test_hd_heats_locally(oracle_lib, kind):
    """What hyper-viscosity/resistivity removes from kinetic/magnetic energy
    reappears as heat: with uniform pressure the local heating rate is
    non-negative everywhere and positive on average (wrong or missing
    v.tau or B x e.m.f. energy-flux terms violate this)."""
    n = 64
    x = W.cell_centres(n, 0.0, 1.0)[None, :]
    if kind == "viscous":
        prob = W.uniform_state(n, 8, v=(0.0, 0.0), b=(0.0, 0.0))
        vy = 0.1 * np.sin(2 * math.pi * x) * np.ones((8, 1))
        prob.fields["my"] = prob.fields["rho"] * vy
        prob.fields["e"] = prob.fields["e"] + 0.5 * prob.fields["rho"] * vy ** 2
    else:
        prob = W.uniform_state(n, 8, v=(0.0, 0.0), b=(0.3, 0.0))
        by = 0.1 * np.sin(2 * math.pi * x) * np.ones((8, 1))
        prob.fields["by"] = by
        prob.fields["e"] = prob.fields["e"] + 0.5 * by ** 2
    K = _hd_only(oracle_lib, prob, 2.0)
    h = _heating(prob, K)
    assert h.mean() > 0
    assert h.min() >= -1e-6 * h.max()
    # heat is deposited where the shear (current) is, i.e. where the profile
    # sin(2 pi x) has its largest slope (x = 0, 1/2), not at its extrema
    # (x = 1/4, 3/4): the heating rate is stress x strain, eta J^2
    row = h[0]
    assert row[[n // 4 - 1, n // 4, 3 * n // 4 - 1, 3 * n // 4]].max() < 0.1 * row[[0, n - 1, n // 2 - 1, n // 2]].min()


def test_shock_term_only_under_compression(oracle_lib):
    """With c2 = 0 only the compression term acts (section 2: diffusion
    becomes large where compression is large): the hyper-diffusive density
    flux vanishes exactly wherever s_f = 0 (expanding flow)."""
    n = 64
    x = W.cell_centres(n, 0.0, 1.0)
    prob = W.uniform_state(n, 1, v=(0.0, 0.0), b=(0.0, 0.0), extent=(1.0, 1.0 / n))
    vx = -0.1 * np.sin(2 * math.pi * x)
    rho = 1.3 * (1 + 0.05 * np.sin(6 * math.pi * x))
    prob.fields["rho"] = rho[None, :].copy()
    prob.fields["mx"] = (rho * vx)[None, :].copy()
    prob.fields["e"] = prob.fields["e"] + 0.5 * (rho * vx ** 2)[None, :]
    K = _hd_only(oracle_lib, prob, 2.0, c2=(0, 0, 0, 0), cshk=(1, 1, 1, 1))[0, 0]
    divv = (np.roll(vx, -1) - np.roll(vx, 1))
    s = np.maximum(0.0, -divv)
    s_face = np.maximum(s, np.roll(s, -1))
    no_flux_cell = (s_face == 0) & (np.roll(s_face, 1) == 0)   # both faces of the cell
    assert no_flux_cell.sum() > 10 and (~no_flux_cell).sum() > 10
    assert np.all(K[no_flux_cell] == 0.0)
    assert np.max(np.abs(K[~no_flux_cell])) > 0


def test_hd_scales_with_max_wave_speed(oracle_lib):
    """Without the compression term the coefficient is proportional to the
    maximum wave speed (section 2)."""
    prob = W.random_smooth(32, 24, seed=2)
    k1 = _hd_only(oracle_lib, prob, 1.0, cshk=(0, 0, 0, 0))
    k3 = _hd_only(oracle_lib, prob, 3.0, cshk=(0, 0, 0, 0))
    assert np.max(np.abs(k3 - 3 * k1)) <= 1e-12 * np.max(np.abs(k3))
    assert np.max(np.abs(k1)) > 0


def _harmonic_case(n=48):
    """Open box, uniform compression v = -a (r - r_c) (so s is uniform) and a
    curl- and divergence-free field B = grad phi, phi = e^{kx} cos(ky) / k^2."""
    prob = W.uniform_state(n, n, v=(0.0, 0.0), b=(0.0, 0.0), bc=(W.problems.OPEN,) * 4)
    x = W.cell_centres(n, 0.0, 1.0)[None, :] * np.ones((n, 1))
    y = W.cell_centres(n, 0.0, 1.0)[:, None] * np.ones((1, n))
    a, k = 0.2, 2.0
    vx, vy = -a * (x - 0.5), -a * (y - 0.5)
    bx = 0.05 * np.exp(k * x) * np.cos(k * y) / k
    by = -0.05 * np.exp(k * x) * np.sin(k * y) / k
    f = prob.fields
    f["mx"], f["my"] = f["rho"] * vx, f["rho"] * vy
    f["bx"], f["by"] = bx, by
    f["e"] = f["e"] + 0.5 * f["rho"] * (vx ** 2 + vy ** 2) + 0.5 * (bx ** 2 + by ** 2)
    return prob


def test_hyper_resistivity_ignores_potential_field(oracle_lib):
    """The hyper-resistive e.m.f. follows the current: with a uniform
    coefficient (c2 = 0, uniform compression) a current-free field is left
    alone up to truncation error, while dropping the cross term is not."""
    prob = _harmonic_case()
    kw = dict(c2=(0, 0, 0, 0), cshk=(1, 1, 1, 1))
    inner = (slice(8, -8), slice(8, -8))
    full = _hd_only(oracle_lib, prob, 1.0, **kw)
    nocross = _hd_only(oracle_lib, prob, 1.0, hd_cross_on=False, **kw)
    big = np.max(np.abs(nocross[5][inner]))
    assert big > 0
    assert np.max(np.abs(full[4][inner])) < 1e-2 * big
    assert np.max(np.abs(full[5][inner])) < 1e-2 * big


def test_hyper_viscosity_stress_is_symmetric(oracle_lib):
    """With a uniform coefficient the stress 1/2 rho nu (d_k v_l + d_l v_k)
    gives 1/2 rho nu (lap v + grad div v): zero for an incompressible flow
    derived from a harmonic stream function (added to a uniform compression)."""
    prob = _harmonic_case()
    f = prob.fields
    n = prob.nx
    x = W.cell_centres(n, 0.0, 1.0)[None, :] * np.ones((n, 1))
    y = W.cell_centres(n, 0.0, 1.0)[:, None] * np.ones((1, n))
    k = 2.0
    wx = 0.05 * np.exp(k * x) * np.cos(k * y)    # d_y psi with psi = e^{kx} sin(ky) / k
    wy = -0.05 * np.exp(k * x) * np.sin(k * y)   # -d_x psi
    rho = f["rho"]
    vx, vy = f["mx"] / rho + wx, f["my"] / rho + wy
    f["e"] = f["e"] - 0.5 * (f["mx"] ** 2 + f["my"] ** 2) / rho + 0.5 * rho * (vx ** 2 + vy ** 2)
    f["mx"], f["my"] = rho * vx, rho * vy
    kw = dict(c2=(0, 0, 0, 0), cshk=(1, 1, 1, 1))
    inner = (slice(8, -8), slice(8, -8))
    full = _hd_only(oracle_lib, prob, 1.0, **kw)
    nocross = _hd_only(oracle_lib, prob, 1.0, hd_cross_on=False, **kw)
    big = max(np.max(np.abs(nocross[1][inner])), np.max(np.abs(nocross[2][inner])))
    assert big > 0
    assert np.max(np.abs(full[1][inner])) < 1e-2 * big
    assert np.max(np.abs(full[2][inner])) < 1e-2 * big
