"""GPU parity of the gravity sources (paper section 2: rho g and rho g.v; in
the split form rho~ g and rho~ g.v) against the FP64 oracle, through the C ABI.

FP64: bit for bit, as every FP64 path (the stage tiles reproduce the oracle's
operation sequence).  FP32: error against the FP64 oracle.
"""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
OPEN = W.problems.OPEN


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _exact(oracle_lib, got, prob, nsteps, label, **kw):
    ora = oracle_lib.State(prob, form=oracle_lib.LOWSTORE, **kw)
    ora.run(nsteps)
    ref = ora.stacked()
    nd = int(np.sum(got != ref))
    errs = [oracle_lib.rel_l2(got[k], ref[k]) for k in range(6)]
    print(f"[gravity] {label}: rel-L2 " + " ".join(f"{e:.1e}" for e in errs) + f"; {nd} elements differ", flush=True)
    assert nd == 0, label
    return ora


@pytest.mark.parametrize("nt", [64, 128])
def test_stratified_atmosphere_parity(oracle_lib, nt):
    """Stratified background (open top and bottom) with a wave pulse under
    gravity: bit for bit."""
    _torch()
    from paper_1710_06423_amd import Solver
    print(f"case: stratified 96x130 launch {nt}", flush=True)
    prob = W.stratified_atmosphere(96, 130, amp=0.05, b_b=(0.1, 0.4))
    s = Solver.from_problem(prob)
    s.set_launch(nt, 0)
    s.advance(25)
    _exact(oracle_lib, s.read_fields().cpu().numpy(), prob, 25, f"stratified launch {nt}")


def test_hydrostatic_atmosphere_stays_static():
    torch = _torch()
    from paper_1710_06423_amd import Solver
    prob = W.stratified_atmosphere(70, 90, amp=0.0, b_b=(0.2, 0.3))
    s = Solver.from_problem(prob)
    s.advance(30)
    assert bool(torch.all(s.read_fields() == 0))


@pytest.mark.parametrize("split", [True, False])
def test_gravity_without_background_parity(oracle_lib, split):
    """Orszag-Tang under gravity, no background: the two FP64 tiles, bit for
    bit (the gravity source with the velocity of the same row)."""
    _torch()
    from paper_1710_06423_amd import Solver
    print(f"case: OT 200x96 gravity split={split}", flush=True)
    prob = W.with_gravity(W.orszag_tang(200, ny=96), (0.4, -0.9))
    s = Solver.from_problem(prob)
    s.set_column_split(split)
    s.advance(20)
    _exact(oracle_lib, s.read_fields().cpu().numpy(), prob, 20, f"OT gravity split={split}")


def test_gravity_one_dimensional_parity(oracle_lib):
    """A Brio-Wu tube with gravity along and across it (1-D tile)."""
    _torch()
    from paper_1710_06423_amd import Solver
    prob = W.with_gravity(W.brio_wu(600), (0.5, -0.3))
    s = Solver.from_problem(prob)
    s.advance(60)
    _exact(oracle_lib, s.read_fields().cpu().numpy(), prob, 60, "BW 600 gravity")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gravity_batch_equals_single_runs(precision):
    """Batched instances with their own gravity evolve exactly as alone."""
    torch = _torch()
    from paper_1710_06423_amd import Batch, Solver, FP32, FP64
    prec = FP32 if precision == "fp32" else FP64
    probs = [W.with_gravity(W.orszag_tang(96, ny=64), (0.0, -1.2)), W.with_gravity(W.brio_wu(400), (0.7, 0.0)),
             W.orszag_tang(80)]
    b = Batch(probs, precision=prec)
    b.advance(15)
    for i, p in enumerate(probs):
        s = Solver.from_problem(p, precision=prec)
        s.advance(15)
        assert torch.equal(b[i].read_fields(), s.read_fields()), i
    b.close()


def test_fp32_stratified_error(oracle_lib):
    """FP32 bulk on a stratified atmosphere (background varying by e^4 over
    the domain): the split perturbations keep a small error against the FP64
    oracle.  Evolving the totals instead (unsplit, same FP32 path) puts the
    background itself under the discrete hydrostatic balance and the
    zero-gradient open boundaries, and the perturbation is lost: the split
    form is what makes this medium tractable."""
    _torch()
    from paper_1710_06423_amd import Solver, FP32
    prob = W.stratified_atmosphere(128, 160, amp=0.05, b_b=(0.1, 0.4))
    ora = oracle_lib.State(prob, form=oracle_lib.LOWSTORE)
    ora.run(40)
    ref = ora.stacked()
    s = Solver.from_problem(prob, precision=FP32)
    s.advance(40)
    split = s.read_fields().cpu().numpy().astype(np.float64)
    # the same state with the background folded into FP32 totals
    f = prob.copy_fields()
    for k, kb in (("rho", "rho_b"), ("e", "e_b"), ("bx", "bx_b"), ("by", "by_b")):
        f[k] = f[k] + prob.background[kb]
    tot = W.Problem("unsplit", prob.nx, prob.ny, prob.x0, prob.x1, prob.y0, prob.y1, prob.gamma, prob.bc, f,
                    None, 0.0, {}, prob.g)
    u = Solver.from_problem(tot, precision=FP32)
    u.advance(40)
    unsplit = u.read_fields().cpu().numpy().astype(np.float64)
    for i, kb in ((0, "rho_b"), (3, "e_b"), (4, "bx_b"), (5, "by_b")):
        unsplit[i] = unsplit[i] - prob.background[kb]
    es = [oracle_lib.rel_l2(split[k], ref[k]) for k in range(4)]
    eu = [oracle_lib.rel_l2(unsplit[k], ref[k]) for k in range(4)]
    print("[gravity] FP32 perturbation rel-L2 (rho~, mx, my, e~): split " + " ".join(f"{e:.2e}" for e in es)
          + "; unsplit " + " ".join(f"{e:.2e}" for e in eu), flush=True)
    assert max(es) < 1e-3
    for k in range(4):
        assert es[k] < eu[k], k
