"""The oracle's two arithmetic forms, and its conservation sums, pinned.

The oracle is defined by its paper form: classic fourth-order Runge-Kutta
(section 2) combined as printed, U+ = U + dt/6 (K1 + 2 K2 + 2 K3 + K4), with
every division of the scheme written as a division.  Its low-storage form is
the same polynomial in dt rearranged onto four state arrays, with reciprocals
of the grid constants, of rho and of gamma - 1.  The device path follows the
low-storage operation sequence, so its bit-exact tests compare with that form;
the tests here tie that form to the definition:

* without hyper-diffusion the scheme does not amplify rounding, and the two
  forms stay within 1e-13 (relative L2, per field) over 60 steps;
* with it, the ratio-of-maxima coefficient amplifies rounding-order
  differences step by step, so they are held within 1e-12 over 3 steps.

The conservation sums (O-10) are pinned to values fixed by the data: exact
sums of dyadic states, row- and column-indexed fields, and the closed-form
integrals of the Orszag-Tang state.
"""

import math

import numpy as np
import pytest

import workloads as W


def _rel_per_field(a, b):
    out = []
    for k in range(a.shape[0]):
        nb = np.sqrt(np.sum(b[k] ** 2))
        d = np.sqrt(np.sum((a[k] - b[k]) ** 2))
        out.append(d / nb if nb > 0 else d)
    return np.array(out)


def _both(oracle_lib, prob, nsteps, **kw):
    p = oracle_lib.State(prob, form=oracle_lib.PAPER, **kw)
    q = oracle_lib.State(prob, form=oracle_lib.LOWSTORE, **kw)
    p.run(nsteps)
    q.run(nsteps)
    return p, q


# ------------------------------------------------------ the paper form

def test_paper_step_is_textbook_rk4(oracle_lib):
    """One step of the paper form equals U + dt/6 (K1 + 2K2 + 2K3 + K4) built
    here from separate right-hand-side evaluations at the textbook stage
    inputs U + dt/2 K1, U + dt/2 K2, U + dt K3 (numpy evaluates the same
    operations in the same order, so the match is exact)."""
    for prob in (W.orszag_tang(48), W.brio_wu(200), W.random_smooth(30, 26, seed=5)):
        s = oracle_lib.State(prob)
        cx, cy, cmax, dt = s.wavespeed()
        cfg = s.cfg
        U = prob.stacked()
        K1 = oracle_lib.rhs(cfg, list(U), None, cmax)
        K2 = oracle_lib.rhs(cfg, list(U + 0.5 * dt * K1), None, cmax)
        K3 = oracle_lib.rhs(cfg, list(U + 0.5 * dt * K2), None, cmax)
        K4 = oracle_lib.rhs(cfg, list(U + dt * K3), None, cmax)
        text = U + dt / 6 * (((K1 + 2 * K2) + 2 * K3) + K4)
        s.run(1)
        assert s.last[0] == dt
        assert np.array_equal(s.stacked(), text)


def test_paper_rhs_divides(oracle_lib):
    """The paper form's right-hand side of a linear profile along x is the
    exact derivative formed by division: for rho~ = a + b x with uniform
    velocity v0 the mass flux is v0 rho~ and L(rho~) = -v0 b wherever the
    stencil does not reach the periodic wrap."""
    n = 40
    prob = W.uniform_state(n, 1, rho=1.0, v=(0.5, 0.0), p=1.0, b=(0.0, 0.0))
    x = W.cell_centres(n, 0.0, 1.0)
    rho = 1.0 + 0.25 * x
    prob.fields["rho"] = rho[None, :].copy()
    prob.fields["mx"] = 0.5 * prob.fields["rho"]
    prob.fields["e"] = 1.0 / (prob.gamma - 1.0) + 0.5 * prob.fields["rho"] * 0.25
    K = oracle_lib.State(prob, hd_on=False).rhs(1.0)
    assert np.max(np.abs(K[0][0, 4:-4] + 0.5 * 0.25)) < 1e-13


# ------------------------------------------ the two forms tied together

@pytest.mark.parametrize("case", ["ot64", "smooth", "entropy", "gravity"])
def test_lowstore_tracks_paper_without_hd(oracle_lib, case):
    """Without hyper-diffusion the low-storage form stays within 1e-13 of the
    paper form over 60 steps, per field."""
    if case == "ot64":
        prob = W.orszag_tang(64)
    elif case == "smooth":
        prob = W.random_smooth(40, 36, seed=2)
    elif case == "entropy":
        prob = W.entropy_wave(48)
    else:
        prob = W.stratified_atmosphere(24, 40)
    p, q = _both(oracle_lib, prob, 60, hd_on=False)
    assert p.steps == q.steps == 60
    assert abs(p.t - q.t) <= 1e-13 * p.t
    err = _rel_per_field(q.stacked(), p.stacked())
    assert np.all(err <= 1e-13), err


@pytest.mark.parametrize("case", ["ot64", "brio_wu", "smooth_nocross", "gravity"])
def test_lowstore_tracks_paper_with_hd(oracle_lib, case):
    """With hyper-diffusion on, the two forms stay within 1e-12 over 3 steps."""
    kw = {}
    if case == "ot64":
        prob = W.orszag_tang(64)
    elif case == "brio_wu":
        prob = W.brio_wu(400)
    elif case == "smooth_nocross":
        prob = W.random_smooth(40, 36, seed=4)
        kw["hd_cross_on"] = False
    else:
        prob = W.stratified_atmosphere(24, 40)
    p, q = _both(oracle_lib, prob, 3, **kw)
    err = _rel_per_field(q.stacked(), p.stacked())
    assert np.all(err <= 1e-12), err


def test_lowstore_rhs_and_speeds_round_like_paper(oracle_lib):
    """One right-hand side and the wave speeds of the two forms agree to a few
    units of rounding (the forms differ only in division against
    multiplication by a reciprocal)."""
    prob = W.random_smooth(30, 34, seed=7)
    p = oracle_lib.State(prob, form=oracle_lib.PAPER)
    q = oracle_lib.State(prob, form=oracle_lib.LOWSTORE)
    wp, wq = np.array(p.wavespeed()), np.array(q.wavespeed())
    assert np.all(np.abs(wp - wq) <= 4e-16 * np.abs(wp))
    Kp, Kq = p.rhs(wp[2]), q.rhs(wp[2])
    for k in range(6):
        scale = np.max(np.abs(Kp[k])) + 1e-300
        assert np.max(np.abs(Kp[k] - Kq[k])) <= 1e-13 * scale


def test_lowstore_keeps_uniform_states_bitwise(oracle_lib):
    """L = 0 leaves a uniform state exactly in place in the low-storage form
    as well: S3 = U and A = 2U, so (A - 2 S3)/3 vanishes."""
    prob = W.uniform_state(12, 10, bc=(1, 1, 0, 0))
    q = oracle_lib.State(prob, form=oracle_lib.LOWSTORE)
    q.run(20)
    assert np.array_equal(q.stacked(), prob.stacked())


@pytest.mark.parametrize("form", ["paper", "lowstore"])
def test_patch_step_matches_full_step_in_each_form(oracle_lib, form):
    """The patch entry point follows the selected form exactly."""
    fm = oracle_lib.PAPER if form == "paper" else oracle_lib.LOWSTORE
    prob = W.random_smooth(44, 40, seed=1)
    s = oracle_lib.State(prob, form=fm)
    cx, cy, cmax, dt = s.wavespeed()
    f0 = s.stacked()
    s.run(1)
    full = s.stacked()
    ii = np.arange(7, 7 + 44) % 44
    jj = np.arange(30, 30 + 40) % 40
    patch = [f0[k][np.ix_(jj, ii)] for k in range(6)]
    out = oracle_lib.step_patch(s.cfg, patch, None, dt, cmax)
    ref = np.stack([full[k][np.ix_(jj[12:-12], ii[12:-12])] for k in range(6)])
    assert np.array_equal(out, ref)


# ------------------------------------------------- conservation sums

def _cfg_for(oracle_lib, nx, ny, x1, y1):
    prob = W.uniform_state(nx, ny, extent=(x1, y1))
    return oracle_lib.make_cfg(prob)


def test_sums_of_dyadic_uniform_state_are_exact(oracle_lib):
    """A uniform dyadic value on a dyadic grid sums exactly to value x area."""
    nx, ny = 64, 32
    cfg = _cfg_for(oracle_lib, nx, ny, 2.0, 1.0)   # dx = dy = 1/32
    vals = [1.5, -0.25, 3.0, 0.0, 2.0 ** -10, 7.75]
    f = [np.full((ny, nx), v) for v in vals]
    got = oracle_lib.sums(cfg, f)
    assert list(got) == [v * 2.0 for v in vals]


def test_sums_see_every_row_and_column_once(oracle_lib):
    """f = row index sums to nx * ny(ny-1)/2 * dx dy; f = column index to
    ny * nx(nx-1)/2 * dx dy; f = 1 on one row only to nx dx dy (all exact
    in binary), so a dropped or doubled row or column, or a transposed
    index, changes the result."""
    nx, ny = 40, 24
    cfg = _cfg_for(oracle_lib, nx, ny, 5.0, 3.0)   # dx = dy = 1/8
    dxdy = (5.0 / nx) * (3.0 / ny)
    jj, ii = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    one_row = np.zeros((ny, nx))
    one_row[ny - 1] = 1.0
    one_col = np.zeros((ny, nx))
    one_col[:, 0] = 1.0
    f = [jj, ii, one_row, one_col, np.ones((ny, nx)), jj * 64.0 + ii]
    got = oracle_lib.sums(cfg, f)
    want = [nx * ny * (ny - 1) / 2 * dxdy, ny * nx * (nx - 1) / 2 * dxdy, nx * dxdy, ny * dxdy,
            nx * ny * dxdy, (64.0 * nx * ny * (ny - 1) / 2 + ny * nx * (nx - 1) / 2) * dxdy]
    assert list(got) == want


def test_sums_of_orszag_tang_match_closed_forms(oracle_lib):
    """On [0, 2pi]^2 the midpoint sums of the Orszag-Tang state are its
    integrals: mass rho (2pi)^2 = 25 pi / 9, zero net momentum and field, and
    energy 4 pi^2 p/(gamma-1) + 2 pi^2 rho + 2 pi^2 B0^2 (the kinetic term
    rho (sin^2 y + sin^2 x)/2 and the magnetic term B0^2 (sin^2 y +
    sin^2 2x)/2 integrate to half their peak times the area)."""
    for n, ny in ((64, 64), (96, 40)):
        prob = W.orszag_tang(n, ny=ny)
        cfg = oracle_lib.make_cfg(prob)
        got = oracle_lib.sums(cfg, [prob.fields[k] for k in W.FIELDS])
        rho = 25.0 / (36.0 * math.pi)
        p = 5.0 / (12.0 * math.pi)
        b0 = 1.0 / math.sqrt(4.0 * math.pi)
        mass = 25.0 * math.pi / 9.0
        energy = 4 * math.pi ** 2 * p / (5.0 / 3.0 - 1.0) + 2 * math.pi ** 2 * rho + 2 * math.pi ** 2 * b0 ** 2
        assert abs(got[0] - mass) <= 1e-13 * mass
        assert abs(got[3] - energy) <= 1e-13 * energy
        for k in (1, 2, 4, 5):
            assert abs(got[k]) <= 1e-13 * mass, (k, got[k])
