"""The device problem generators (sacx_init_problem; paper section 5, the
Orszag-Tang vortex and the Brio-Wu shock tube) against the host generators
of the workloads, and runs from the generated states against the oracle."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _blank(prob, precision=0):
    """A context with the problem's grid and parameters, nothing loaded."""
    from paper_1710_06423_amd import Solver
    return Solver.from_problem(prob, precision=precision, init=False)


@pytest.mark.parametrize("n,ny,b0", [(200, 136, ()), (96, 96, (1.3,))])
def test_orszag_tang_generator(oracle_lib, n, ny, b0):
    """Within the last bit of the host evaluation (the sines), exact
    elsewhere; a run from the generated state follows the oracle run from
    that same state bit for bit."""
    torch = _torch()
    from paper_1710_06423_amd import PROBLEM_ORSZAG_TANG
    prob = W.orszag_tang(n, ny=ny, b0_scale=b0[0] if b0 else 1.0)
    s = _blank(prob)
    s.set_boundaries((1, 1, 1, 1))          # the generator sets the problem's own
    s.init_problem(PROBLEM_ORSZAG_TANG, b0)
    got = s.read_fields().cpu().numpy()
    ref = prob.stacked()
    assert np.array_equal(got[0], ref[0])
    for k in range(1, 6):
        scale = np.abs(ref[k]).max()
        assert np.abs(got[k] - ref[k]).max() <= 4e-16 * scale, k
    print(f"[init] OT {n}x{ny}: {int((got != ref).sum())} of {got.size} values differ from the host's in the last bit",
          flush=True)
    s.advance(12)
    run = W.Problem("ot_device", prob.nx, prob.ny, prob.x0, prob.x1, prob.y0, prob.y1, prob.gamma, prob.bc,
                    {k: got[i].copy() for i, k in enumerate(W.FIELDS)}, None, 0.0, {}, prob.g)
    ora = oracle_lib.State(run, form=oracle_lib.LOWSTORE)
    ora.run(12)
    assert np.array_equal(s.read_fields().cpu().numpy(), ora.stacked())


@pytest.mark.parametrize("n,scales,along_y", [(800, (), False), (513, (1.7, 0.6), False), (400, (0.8,), True)])
def test_brio_wu_generator_bit_exact(oracle_lib, n, scales, along_y):
    """No transcendental: the generated tube equals the host's bit for bit,
    and so does the run (open ends set by the generator)."""
    torch = _torch()
    from paper_1710_06423_amd import PROBLEM_BRIO_WU
    sl = scales[0] if len(scales) > 0 else 1.0
    sr = scales[1] if len(scales) > 1 else 1.0
    prob = W.brio_wu(n, sl, sr, along_y=along_y)
    s = _blank(prob)
    s.set_boundaries((0, 0, 0, 0))
    s.init_problem(PROBLEM_BRIO_WU, scales)
    assert np.array_equal(s.read_fields().cpu().numpy(), prob.stacked())
    s.advance(30)
    ora = oracle_lib.State(prob, form=oracle_lib.LOWSTORE)
    ora.run(30)
    assert np.array_equal(s.read_fields().cpu().numpy(), ora.stacked())


def test_two_dimensional_tube_and_fp32():
    """A 2-D grid gets the tube along x in every row; an FP32 context gets
    the FP64 values rounded once."""
    torch = _torch()
    from paper_1710_06423_amd import FP32, PROBLEM_BRIO_WU, PROBLEM_ORSZAG_TANG
    prob = W.brio_wu(64)
    s = _blank(W.Problem("tube2d", 64, 5, 0.0, 1.0, 0.0, 0.5, 2.0, prob.bc, prob.fields, None, 0.0, {}, (0.0, 0.0)))
    s.init_problem(PROBLEM_BRIO_WU)
    got = s.read_fields().cpu().numpy()
    assert np.array_equal(got, np.repeat(prob.stacked(), 5, axis=1))
    ot = W.orszag_tang(64)
    f32 = _blank(ot, precision=FP32)
    f32.init_problem(PROBLEM_ORSZAG_TANG)
    a = f32.read_fields(torch.float32).cpu().numpy()
    b = ot.stacked().astype(np.float32)
    assert np.abs(a.astype(np.float64) - b).max() <= 2 * np.finfo(np.float32).eps


def test_generator_rejects_bad_requests():
    torch = _torch()
    from paper_1710_06423_amd import PROBLEM_BRIO_WU, PROBLEM_ORSZAG_TANG, SacxError, sacx
    s = _blank(W.orszag_tang(32))
    for kind, prm in ((7, ()), (PROBLEM_ORSZAG_TANG, (1.0, 2.0)), (PROBLEM_BRIO_WU, (0.0,)),
                      (PROBLEM_BRIO_WU, (1.0, float("nan"))), (PROBLEM_BRIO_WU, (1.0, 1.0, 1.0))):
        with pytest.raises(SacxError) as e:
            s.init_problem(kind, prm)
        assert e.value.code == sacx.EINVAL, (kind, prm)
    bg = _blank(W.stratified_atmosphere(16, 20))
    with pytest.raises(SacxError) as e:
        bg.init_problem(PROBLEM_ORSZAG_TANG)
    assert e.value.code == sacx.EUNSUP
