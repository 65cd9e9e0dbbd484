"""Pins of the oracle's gravity terms (paper section 2: the momentum source
rho g and the energy source rho g.v; in the split form the background is in
equilibrium under its own pressure and field, leaving rho~ g and rho~ g.v).

Each pin is fixed by something other than the formula itself: an exact
equilibrium, a closed-form solution RK4 integrates without truncation error,
the discrete pressure gradient of the unsplit form, a momentum budget, and
the x <-> y symmetry.
"""

import math

import numpy as np
import pytest

import workloads as W

OPEN = W.problems.OPEN


@pytest.mark.parametrize("b_b,hd_on", [((0.0, 0.0), True), ((0.3, 0.6), True), ((0.3, 0.6), False)])
def test_hydrostatic_atmosphere_stays_static_bitwise(oracle_lib, b_b, hd_on):
    """A stratified background in hydrostatic equilibrium with no perturbation
    is an exact steady state of the split form: every perturbation field stays
    exactly zero (gravity acting on the total density would push it)."""
    prob = W.stratified_atmosphere(24, 40, b_b=b_b, amp=0.0)
    s = oracle_lib.State(prob, hd_on=hd_on)
    s.run(30)
    assert s.steps == 30
    for k, v in s.fields().items():
        assert np.array_equal(v, np.zeros_like(v)), k


@pytest.mark.parametrize("rho_b_frac", [0.0, 0.5])
def test_uniform_acceleration_closed_form(oracle_lib, rho_b_frac):
    """A uniform state under uniform gravity stays uniform; with rho~ the
    perturbation density and rho the total, m(t) = m0 + rho~ g t (linear) and
    e(t) = e0 + (rho~/rho)(g.m0 t + rho~ |g|^2 t^2 / 2) (quadratic), both of
    which classic RK4 integrates exactly, whatever the time steps."""
    g = (0.3, -0.5)
    base = W.uniform_state(12, 10)
    rho = float(base.fields["rho"][0, 0])
    if rho_b_frac:
        e_b = 0.4
        prob = W.split_background(base, rho * rho_b_frac, e_b, (0.0, 0.0))
    else:
        prob = base
    prob = W.with_gravity(prob, g)
    rt = float(prob.fields["rho"][0, 0])
    m0 = np.array([prob.fields["mx"][0, 0], prob.fields["my"][0, 0]])
    e0 = float(prob.fields["e"][0, 0])
    s = oracle_lib.State(prob)
    s.run(25)
    t = s.t
    f = s.fields()
    for k, v in f.items():
        assert np.all(v == v.flat[0]), k   # still uniform, bit for bit
    gv = np.array(g)
    m_ref = m0 + rt * gv * t
    e_ref = e0 + (rt / rho) * (float(gv @ m0) * t + rt * float(gv @ gv) * t * t / 2)
    assert abs(f["mx"][0, 0] - m_ref[0]) <= 1e-13 * max(1.0, abs(m_ref[0]))
    assert abs(f["my"][0, 0] - m_ref[1]) <= 1e-13 * max(1.0, abs(m_ref[1]))
    assert abs(f["e"][0, 0] - e_ref) <= 1e-13 * max(1.0, abs(e_ref))
    assert f["rho"][0, 0] == rt


def _unsplit_imbalance(oracle_lib, n, t_end):
    """Largest interior |m_y| after t_end of the hydrostatic atmosphere run in
    the unsplit form (background folded into the evolved fields), HD off."""
    p = W.stratified_atmosphere(8, n, amp=0.0)
    f = p.copy_fields()
    f["rho"] = f["rho"] + p.background["rho_b"]
    f["e"] = f["e"] + p.background["e_b"]
    q = W.Problem("unsplit", p.nx, p.ny, p.x0, p.x1, p.y0, p.y1, p.gamma, p.bc, f, None, 0.0, {}, p.g)
    s = oracle_lib.State(q, hd_on=False)
    s.run(100000, t_end)
    my = s.fields()["my"]
    y = W.cell_centres(n, p.y0, p.y1)
    inner = (y > 0.35) & (y < 0.65)
    return float(np.max(np.abs(my[inner, :])))


def test_unsplit_hydrostatic_balance_converges_fourth_order(oracle_lib):
    """In the unsplit form the hydrostatic balance is discrete: the
    fourth-order pressure gradient against rho g leaves an O(h^4) force, so the
    spurious interior momentum falls ~16x per halving of h (a wrong sign or
    component of the gravity source would leave an O(1) imbalance)."""
    t_end = 0.05
    a = _unsplit_imbalance(oracle_lib, 40, t_end)
    b = _unsplit_imbalance(oracle_lib, 80, t_end)
    print(f"[gravity] unsplit imbalance |m_y| {a:.3e} (n=40) -> {b:.3e} (n=80), ratio {a / b:.1f}")
    assert a < 1e-5
    assert a / b > 12.0


def test_momentum_budget_periodic(oracle_lib):
    """On a periodic domain the fluxes cancel in the sums, so
    sum m(t) = sum m(0) + g sum(rho~) t, with sum(rho~) conserved."""
    g = (0.2, -0.7)
    prob = W.with_gravity(W.orszag_tang(32), g)
    s = oracle_lib.State(prob)
    s0 = s.sums().copy()
    s.run(30)
    s1 = s.sums()
    t = s.t
    assert abs(s1[0] - s0[0]) <= 1e-13 * abs(s0[0])
    for k, gk in ((1, g[0]), (2, g[1])):
        ref = s0[k] + gk * s0[0] * t
        assert abs(s1[k] - ref) <= 1e-12 * max(1.0, abs(gk * s0[0] * t)), (k, s1[k], ref)


def test_transpose_with_gravity_bitwise(oracle_lib):
    """x <-> y exchange (fields, boundaries and the gravity vector) commutes
    with the scheme, sources included, bit for bit."""
    p = W.with_gravity(W.random_smooth(24, 18, seed=11), (0.3, -0.6))
    q = W.transpose_problem(p)
    assert q.g == (-0.6, 0.3)
    a, b = oracle_lib.State(p), oracle_lib.State(q)
    a.run(15)
    b.run(15)
    fa, fb = a.fields(), b.fields()
    for ka, kb in (("rho", "rho"), ("mx", "my"), ("my", "mx"), ("e", "e"), ("bx", "by"), ("by", "bx")):
        assert np.array_equal(fa[ka], fb[kb].T), ka


def test_stratified_pulse_front_moves_at_sound_speed(oracle_lib):
    """The stratified-atmosphere workload (isothermal, so the sound speed
    c_s = sqrt(gamma g H) is the same at every height): the upper front of the
    velocity pulse moves up at about c_s, the perturbation density becomes
    non-zero (so the gravity source acts), and the totals stay positive."""
    prob = W.stratified_atmosphere(32, 64, amp=0.05)
    cs = math.sqrt(prob.gamma * prob.meta["g0"] * prob.meta["H"])
    y = W.cell_centres(prob.ny, prob.y0, prob.y1)

    def front(f):
        vy = f["my"] / (f["rho"] + prob.background["rho_b"])
        col = np.abs(vy).max(axis=1)
        return y[np.nonzero(col > 0.01 * prob.meta["amp"] * cs)[0].max()]

    t_end = 0.2
    s = oracle_lib.State(prob)
    s.run(100000, t_end)
    f = s.fields()
    assert np.all(f["rho"] + prob.background["rho_b"] > 0) and np.all(np.isfinite(f["e"]))
    assert np.max(np.abs(f["rho"])) > 0.0
    speed = (front(f) - front(prob.fields)) / t_end
    print(f"[gravity] pulse front speed {speed:.3f}, c_s {cs:.3f}")
    assert 0.7 * cs < speed < 1.3 * cs
