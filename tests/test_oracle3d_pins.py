"""Pins of the 3-D oracle (oracle/sacx_oracle3d.c) against things other than
itself: the pinned 2-D oracle bit for bit in every plane, uniform states,
the oblique entropy wave's convergence order, conservation, div B, and the
symmetry of the scheme under permutations and reflections of the axes."""

import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import oracle3d as O3


@pytest.fixture(scope="module", autouse=True)
def _built():
    O3.build(force=False)


def _two_d_cases():
    return [
        ("orszag_tang", W.orszag_tang(24, ny=20)),
        ("brio_wu", W.brio_wu(60)),
        ("random_open", W.random_smooth(18, 22, seed=3, bc=(oracle.OPEN,) * 4)),
        ("random_mixed", W.random_smooth(20, 16, seed=5, bc=(oracle.OPEN, oracle.OPEN, oracle.PERIODIC,
                                                              oracle.PERIODIC))),
    ]


@pytest.mark.parametrize("form", [oracle.PAPER, oracle.LOWSTORE])
@pytest.mark.parametrize("plane", ["xy", "xz", "yz"])
@pytest.mark.parametrize("cross", [True, False])
def test_reduces_bitwise_to_the_2d_oracle_in_every_plane(form, plane, cross):
    """A state that does not vary along one axis and has no velocity or
    field along it evolves, in every layer, exactly as the 2-D oracle's run
    of that plane (3-D sums are ordered so that the vanishing terms drop out
    exactly): fluxes, differences, coefficients, cross terms, boundaries,
    time step and RK4 are all checked against the 2-D definitions."""
    for name, prob in _two_d_cases():
        ref = oracle.State(prob, form=form, hd_cross_on=cross)
        ref.advance(6)
        want = np.stack(ref.f)
        for depth in (1, 3):
            s3 = O3.State3(W.embed_2d(prob, plane, depth=depth), form=form, hd_cross_on=cross)
            s3.run(6)
            assert s3.t == ref.t, (name, depth)
            for layer in range(depth):
                got = W.extract_2d(s3.f, plane, layer)
                assert np.array_equal(got, want), (name, plane, depth, layer, np.abs(got - want).max())
            # the components along the third axis stay exactly zero
            third = {"xy": (3, 7), "xz": (2, 6), "yz": (1, 5)}[plane]
            assert not np.any(s3.f[third[0]]) and not np.any(s3.f[third[1]])


@pytest.mark.parametrize("bc", [(O3.PERIODIC,) * 6, (O3.OPEN,) * 6,
                                (O3.OPEN, O3.OPEN, O3.PERIODIC, O3.PERIODIC, O3.OPEN, O3.OPEN)])
def test_uniform_state_stays_bitwise_uniform(bc):
    """Every difference of a uniform state is zero, the coefficient ratio is
    0 where the first differences vanish, so L = 0 and RK4 keeps the state
    bit for bit (paper form), with every velocity and field component
    non-zero and hyper-diffusion on."""
    prob = W.uniform_3d(9, 7, 8, bc=bc)
    s = O3.State3(prob)
    s.run(12)
    assert s.steps == 12
    assert np.array_equal(s.f, prob.stacked())
    low = O3.State3(prob, form=O3.LOWSTORE)
    low.run(12)
    # the low-storage combine (A + w3)/3 rounds: a uniform state moves by ulps
    assert np.max(np.abs(low.f - prob.stacked())) <= 1e-14 * np.max(np.abs(prob.stacked()))


def _entropy_error(n: int, t_end: float) -> float:
    prob = W.entropy_wave_3d(n)
    s = O3.State3(prob, hd_on=False)
    s.run(100000, t_end=t_end)
    exact = W.entropy_wave_3d_exact(n, s.t)
    return float(np.sqrt(np.mean((s.f[0] - exact) ** 2)))


def test_oblique_entropy_wave_converges_at_fourth_order():
    """The density profile advected obliquely along (1, 1, 1) with uniform
    v, p and B is an exact non-linear solution; the error against it falls
    at fourth order in the cell size (HD off): differences along all three
    axes and the RK4 combine."""
    t_end = 0.05
    errs = [_entropy_error(n, t_end) for n in (12, 24)]
    order = math.log2(errs[0] / errs[1])
    print("[entropy 3-D] errors", errs, "order", order)
    assert order >= 3.9


def test_conservation_periodic_with_hyper_diffusion():
    """Every term is in flux form: over a periodic box the sums of the
    eight conserved fields stay constant to rounding (cross terms on)."""
    prob = W.random_smooth_3d(12, 10, 14, seed=4)
    s = O3.State3(prob)
    s0 = s.sums()
    s.run(8)
    s1 = s.sums()
    scale = np.array([np.sum(np.abs(prob.stacked()[k])) for k in range(8)]) * np.prod(prob.h)
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s1 - s0) / scale


def _div_b(f, h):
    """Fourth-order central divergence of B on a periodic box."""
    def d(a, axis, hh):
        return (8.0 * (np.roll(a, -1, axis) - np.roll(a, 1, axis)) - (np.roll(a, -2, axis) - np.roll(a, 2, axis))) / (
            12.0 * hh)
    return d(f[5], 2, h[0]) + d(f[6], 1, h[1]) + d(f[7], 0, h[2])


def test_discrete_div_b_stays_zero_without_hyper_diffusion():
    """The induction fluxes are antisymmetric (F_d(B_k) = -F_k(B_d)) and the
    difference operators commute, so the discrete divergence of B keeps its
    initial value, zero for the 3-D vortex, to rounding."""
    prob = W.orszag_tang_3d(16)
    h = prob.h
    assert np.max(np.abs(_div_b(prob.stacked(), h))) <= 1e-13
    s = O3.State3(prob, hd_on=False)
    s.run(10)
    bmax = np.max(np.abs(s.f[5:8]))
    assert np.max(np.abs(_div_b(s.f, h))) <= 1e-12 * bmax / min(h)


def _permute(f, perm):
    """Relabel the axes: new axis perm[a] holds old axis a (fields and
    vector components follow)."""
    # numpy axes of a field: z -> 0, y -> 1, x -> 2
    src_axes = [2 - perm.index(a) for a in (2, 1, 0)]
    out = np.empty_like(f)
    for q in (0, 4):
        out[q] = np.transpose(f[q], src_axes)
    for base in (1, 5):
        for a in range(3):
            out[base + perm[a]] = np.transpose(f[base + a], src_axes)
    return out


@pytest.mark.parametrize("perm", [(1, 2, 0), (2, 0, 1), (1, 0, 2)])
def test_right_hand_side_commutes_with_axis_permutations(perm):
    """Relabelling the axes of a cube relabels L: each direction's fluxes,
    coefficients and cross terms are checked against the others' (only the
    order of the sums over directions changes, so to rounding)."""
    prob = W.random_smooth_3d(10, 10, 10, seed=7)
    cfg = O3.make_cfg(prob)
    f = prob.stacked()
    k = O3.rhs(cfg, f, 2.5)
    kp = O3.rhs(cfg, _permute(f, perm), 2.5)
    want = _permute(k, perm)
    scale = np.max(np.abs(k), axis=(1, 2, 3), keepdims=True)
    assert np.max(np.abs(kp - want) / scale) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_right_hand_side_commutes_with_reflections(axis):
    """Mirroring one axis (x -> -x, its velocity and field components change
    sign) mirrors L: signs and one-sided index ranges of every face term."""
    prob = W.random_smooth_3d(11, 9, 10, seed=8)
    cfg = O3.make_cfg(prob)
    f = prob.stacked()
    npax = 2 - axis

    def mirror(a):
        m = np.flip(a, axis=npax + 1).copy()
        m[1 + axis] *= -1.0
        m[5 + axis] *= -1.0
        return m

    k = O3.rhs(cfg, f, 2.5)
    km = O3.rhs(cfg, mirror(f), 2.5)
    scale = np.max(np.abs(k), axis=(1, 2, 3), keepdims=True)
    assert np.max(np.abs(km - mirror(k)) / scale) <= 1e-12


def test_wave_speeds_and_time_step_of_a_uniform_state():
    """c_d = |v_d| + sqrt((gamma p + |B|^2)/rho), dt = CFL min h_d / c_d,
    for a uniform state with the primitives chosen so that the fast speed
    is a round number: gamma p = 1.75, |B|^2 = 2.25, rho = 1 -> c_f = 2."""
    gamma = 1.75
    prob = W.uniform_3d(6, 5, 4, rho=1.0, v=(0.5, -1.25, 0.0), p=1.0, b=(1.0, 1.0, 0.5), gamma=gamma,
                        extent=(0.0, 1.2, 0.0, 1.0, 0.0, 0.8))
    cx, cy, cz, cmax, dt = O3.wavespeed(O3.make_cfg(prob), prob.stacked())
    # (e is formed from the primitives in floating point: to rounding)
    assert (cx, cy, cz, cmax) == pytest.approx((2.5, 3.25, 2.0, 3.25), rel=1e-15)
    assert dt == pytest.approx(0.3 * min(0.2 / 2.5, 0.2 / 3.25, 0.2 / 2.0), rel=1e-15)


def test_non_physical_state_is_refused():
    prob = W.uniform_3d(5, 5, 5)
    f = prob.stacked()
    f[4][2, 2, 2] = -1.0   # energy below the kinetic and magnetic parts: p < 0
    with pytest.raises(RuntimeError):
        O3.wavespeed(O3.make_cfg(prob), f)


def test_sums_of_a_uniform_box_are_value_times_volume():
    prob = W.uniform_3d(6, 5, 4, extent=(0.0, 1.2, 0.0, 1.0, 0.0, 0.8))
    got = O3.sums(O3.make_cfg(prob), prob.stacked())
    want = np.array([prob.stacked()[k][0, 0, 0] for k in range(8)]) * (1.2 * 1.0 * 0.8)
    assert np.allclose(got, want, rtol=1e-14, atol=0.0)


def test_sums_of_the_3d_vortex_in_closed_form():
    """Over a periodic cell-centred grid the mean of sin^2 is 1/2 and of sin
    is 0: mass = rho0 (2 pi)^3, momentum and field sums 0, energy =
    (2 pi)^3 (p/(gamma-1) + rho0 (1 + eps^2)/2 + B0^2/2)."""
    eps = 0.2
    prob = W.orszag_tang_3d(16, eps=eps)
    s = O3.sums(O3.make_cfg(prob), prob.stacked())
    vol = (2.0 * math.pi) ** 3
    rho0, p0, gamma = 25.0 / (36.0 * math.pi), 5.0 / (12.0 * math.pi), 5.0 / 3.0
    b0 = 1.0 / math.sqrt(4.0 * math.pi)
    assert s[0] == pytest.approx(rho0 * vol, rel=1e-13)
    assert s[4] == pytest.approx(vol * (p0 / (gamma - 1.0) + 0.5 * rho0 * (1.0 + eps * eps) + 0.5 * b0 * b0), rel=1e-13)
    for q in (1, 2, 3, 5, 6, 7):
        assert abs(s[q]) <= 1e-13 * vol
