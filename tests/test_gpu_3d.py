"""GPU parity of the three-dimensional scheme: the HIP path (sacx3_* through
the C ABI) against the 3-D FP64 CPU oracle's low-storage form, bit for bit
(the oracle itself is pinned by tests/test_oracle3d_pins.py to the 2-D
oracle in every plane, to closed forms and to invariants).

Sizes span several 32 x 8 column tiles and z strips with ragged tails, both
boundary kinds, the cross terms on and off and hyper-diffusion off.
"""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def O3():
    from oracle import oracle3d
    oracle3d.build(force=False)
    return oracle3d


def _gpu(prob, nsteps, planes=0, **kw):
    _torch()
    from paper_1710_06423_amd.sacx3 import Solver3
    s = Solver3.from_problem(prob, **kw)
    if planes:
        s.set_launch(planes)
    done, t = s.advance(nsteps)
    out = s.read_fields().cpu().numpy()
    return s, out, done, t


def _assert_same(got, ref, label):
    ndiff = int(np.sum(got != ref))
    worst = float(np.max(np.abs(got - ref)))
    print(f"[3d parity] {label}: elements differing {ndiff} of {ref.size}, max |diff| {worst:.3e}", flush=True)
    assert ndiff == 0, (label, ndiff, worst)


def _case(O3, prob, nsteps, label, planes=0, **kw):
    print(f"case: {label} {prob.nx}x{prob.ny}x{prob.nz} steps={nsteps} {kw}", flush=True)
    s, got, done, t = _gpu(prob, nsteps, planes=planes, **kw)
    ref = O3.State3(prob, form=O3.LOWSTORE, **kw)
    ref.run(nsteps)
    assert done == nsteps
    assert t == ref.t, (label, t, ref.t)
    _assert_same(got, ref.f, label)
    return s, got, ref


def test_orszag_tang_3d_48_bit_exact(O3):
    """The 3-D Orszag-Tang vortex at 48^3, periodic, 8 steps."""
    s, got, ref = _case(O3, W.orszag_tang_3d(48), 8, "OT3D 48^3")
    d = s.diagnostics()
    c = O3.wavespeed(ref.cfg, ref.f)
    assert tuple(d["c"]) == c[:3] and d["c_max"] == c[3]
    s.close()


def test_orszag_tang_3d_160_bit_exact(O3):
    """160^3 (5 x 20 tiles, 3 z strips of 64 planes, ragged), 2 steps."""
    s, _, _ = _case(O3, W.orszag_tang_3d(160), 2, "OT3D 160^3")
    s.close()


@pytest.mark.parametrize("bc,label", [
    ((1, 1, 0, 0, 1, 1), "open x and z"),
    ((1,) * 6, "all open"),
    ((0, 0, 1, 1, 0, 0), "open y"),
])
def test_ragged_open_boundaries_bit_exact(O3, bc, label):
    """A smooth random state on a ragged 37 x 21 x 19 grid with open
    (zero-gradient) boundaries, 6 steps."""
    prob = W.random_smooth_3d(37, 21, 19, seed=7, bc=bc)
    s, _, _ = _case(O3, prob, 6, "random " + label)
    s.close()


def test_open_48_bit_exact(O3):
    """48^3 with open boundaries in x and z, periodic in y, 6 steps."""
    prob = W.random_smooth_3d(48, 48, 48, seed=11, bc=(1, 1, 0, 0, 1, 1))
    s, _, _ = _case(O3, prob, 6, "random 48^3 open x,z")
    s.close()


@pytest.mark.parametrize("hd_on,cross", [(True, False), (False, True)])
def test_switches_bit_exact(O3, hd_on, cross):
    """Cross terms off; hyper-diffusion off (the ideal scheme), 5 steps."""
    prob = W.random_smooth_3d(40, 18, 27, seed=2, bc=(0, 0, 1, 1, 0, 0))
    s, _, _ = _case(O3, prob, 5, f"hd={hd_on} cross={cross}", hd_on=hd_on, hd_cross_on=cross)
    s.close()


@pytest.mark.parametrize("planes", [1, 5, 64, 200])
def test_launch_shape_does_not_change_bits(O3, planes):
    """Strip heights along z from 1 plane to more than the grid."""
    prob = W.random_smooth_3d(33, 9, 23, seed=4)
    s, _, _ = _case(O3, prob, 3, f"planes={planes}", planes=planes)
    s.close()


@pytest.mark.parametrize("shape", [(40, 30, 1), (1, 24, 20), (26, 1, 17)])
def test_one_cell_directions_bit_exact(O3, shape):
    """A direction with one cell (periodic; its differences vanish)."""
    nx, ny, nz = shape
    bc = tuple(0 if n == 1 else 1 for n in (nx, nx, ny, ny, nz, nz))
    prob = W.random_smooth_3d(nx, ny, nz, seed=9, bc=bc)
    s, _, _ = _case(O3, prob, 4, f"shape {shape}")
    s.close()


def test_uniform_state_stays_bitwise_uniform():
    """Every difference vanishes, R = 0 where the first differences do: the
    low-storage combine keeps U exactly (L = 0 gives A = 2U and U+ = U)."""
    prob = W.uniform_3d(35, 12, 19, bc=(1, 1, 0, 0, 1, 1))
    s, got, done, _ = _gpu(prob, 10)
    assert done == 10
    assert np.array_equal(got, prob.stacked())
    s.close()


def test_conservation_sums_match_oracle(O3):
    """FP64 sums of the eight fields times the cell volume, against the
    oracle's sums of the same state (summation order differs: 1e-13)."""
    prob = W.orszag_tang_3d(40)
    s, got, _, _ = _gpu(prob, 3)
    d = s.diagnostics()
    ref = O3.sums(O3.make_cfg(prob), got)
    for k in range(8):
        scale = max(abs(ref[k]), 1e-300)
        assert abs(d["sums"][k] - ref[k]) <= 1e-13 * scale + 1e-15, (k, d["sums"][k], ref[k])
    s.close()


def test_embedded_2d_equals_2d_library_run():
    """A 2-D Orszag-Tang problem laid into the xz plane of a 3-D grid steps,
    layer for layer, exactly as the 2-D library path steps the 2-D problem."""
    torch = _torch()
    from paper_1710_06423_amd import Solver
    prob2 = W.orszag_tang(64, ny=48)
    s2 = Solver.from_problem(prob2)
    s2.advance(5)
    want = s2.read_fields().cpu().numpy()
    s2.close()
    prob3 = W.embed_2d(prob2, "xz", depth=3)
    s3, got, done, _ = _gpu(prob3, 5)
    for layer in range(3):
        assert np.array_equal(W.extract_2d(got, "xz", layer), want), layer
    s3.close()


def test_nonphysical_state_stops_stepping():
    """A negative pressure in the start state: no step is taken."""
    torch = _torch()
    from paper_1710_06423_amd import sacx as S
    from paper_1710_06423_amd.sacx3 import Solver3
    prob = W.random_smooth_3d(16, 16, 16, seed=1)
    prob.fields["e"][3, 4, 5] = -1.0
    s = Solver3.from_problem(prob)
    rc, done, t = s.advance_rc(5)
    assert rc == S.ENONPHYS and done == 0 and t == 0.0
    assert s.diagnostics()["nonphys"] == 1
    s.close()


def test_resume_is_bitwise():
    """advance(a + b) equals advance(a), read, init, advance(b)."""
    torch = _torch()
    from paper_1710_06423_amd.sacx3 import Solver3
    prob = W.orszag_tang_3d(24, ny=20, nz=18)
    s = Solver3.from_problem(prob)
    s.advance(6)
    whole = s.read_fields().cpu().numpy()
    s.close()
    a = Solver3.from_problem(prob)
    _, t = a.advance(2)
    mid = a.read_fields()
    a.close()
    b = Solver3.from_problem(prob, init=False)
    b.init_state(mid, t0=t)
    b.advance(4)
    assert np.array_equal(b.read_fields().cpu().numpy(), whole)
    b.close()
