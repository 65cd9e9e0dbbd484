"""Batched persistent launch: every instance must evolve exactly as it does
alone (bit for bit, any precision, any tile shape), and FP64 instances match
the oracle bit for bit."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _mixed(n_bw=3, n_ot=3, seed=5, small=True):
    probs = W.batch_instances(seed=seed, n_bw=n_bw, n_ot=n_ot)
    if small:
        # keep the single-run comparison quick: shrink the boxes, keep the draws
        out = []
        for p in probs:
            if p.ny == 1:
                out.append(W.brio_wu(min(p.nx, 900), p.meta["s_left"], p.meta["s_right"]))
            else:
                out.append(W.orszag_tang(min(p.nx, 200), b0_scale=p.meta["b0"] * np.sqrt(4 * np.pi)))
        probs = out
    return probs


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_single_runs(precision):
    _torch()
    from paper_1710_06423_amd import Batch, Solver, FP32, FP64
    prec = FP32 if precision == "fp32" else FP64
    probs = _mixed()
    print(f"case: batch of {len(probs)} {precision}", flush=True)
    b = Batch(probs, precision=prec)
    b.advance(15)
    for i, p in enumerate(probs):
        s = Solver.from_problem(p, precision=prec)
        s.advance(15)
        a, c = b[i].read_fields().cpu().numpy(), s.read_fields().cpu().numpy()
        nd = int(np.sum(a != c))
        print(f"[batch] instance {i} {p.nx}x{p.ny}: elements differing from the single run {nd}", flush=True)
        assert nd == 0
        assert b[i].diagnostics()["t"] == s.diagnostics()["t"]


def test_batch_fp64_matches_oracle(oracle_lib):
    _torch()
    from paper_1710_06423_amd import Batch, FP64
    probs = [W.brio_wu(500, 1.3, 0.7), W.orszag_tang(160, ny=96), W.brio_wu(300)]
    print("case: fp64 batch vs oracle", flush=True)
    b = Batch(probs, precision=FP64)
    b.advance(12)
    for i, p in enumerate(probs):
        ora = oracle_lib.State(p, form=oracle_lib.LOWSTORE)
        ora.run(12)
        got = b[i].read_fields().cpu().numpy()
        assert np.array_equal(got, ora.stacked()), i
        assert b[i].diagnostics()["t"] == ora.t


def test_batch_tile_shapes_do_not_change_results():
    torch = _torch()
    from paper_1710_06423_amd import Batch, FP32
    probs = _mixed(2, 2, seed=9)
    outs = []
    for threads, rows in ((128, 16), (256, 64), (64, 7)):
        b = Batch(probs, precision=FP32)
        b.set_tiles(threads, [rows] * len(probs))
        b.advance(6)
        outs.append([b[i].read_fields() for i in range(len(probs))])
    for k in range(1, len(outs)):
        for i in range(len(probs)):
            assert torch.equal(outs[0][i], outs[k][i]), (k, i)


def test_batch_requires_initialised_instances():
    _torch()
    from paper_1710_06423_amd import Batch, FP32, sacx
    b = Batch(_mixed(1, 1), precision=FP32, init=False)
    with pytest.raises(sacx.SacxError) as e:
        b.advance(1)
    assert e.value.code == sacx.ESTATE


@pytest.mark.slow
def test_batch_64_mixed_workload(oracle_lib):
    """The 64-instance mixed workload (32 shock tubes N in [400, 3200], 32
    vortex boxes side in [128, 768]), FP32 bulk, 100 steps: sampled instances
    are bit-identical to their single runs; FP32 error vs the FP64 oracle is
    reported per instance for a sample."""
    _torch()
    from paper_1710_06423_amd import Batch, Solver, FP32
    from paper_1710_06423_amd.autotune import tune_batch
    probs = W.batch_instances(seed=0)
    print("case: batch 64 fp32 100 steps", flush=True)
    b = Batch(probs, precision=FP32)
    t, r, _ = tune_batch(b, use_cache=False, steps=1)
    for i in range(len(probs)):          # restart from the initial states after tuning
        import torch
        f = torch.stack([torch.from_numpy(probs[i].fields[k]) for k in W.FIELDS]).to(b.device)
        b[i].init_state(f)
    b.advance(100)
    for i in (0, 7, 31, 32, 40, 63):
        s = Solver.from_problem(probs[i], precision=FP32)
        s.advance(100)
        a, c = b[i].read_fields().cpu().numpy(), s.read_fields().cpu().numpy()
        assert np.array_equal(a, c), i
    # FP32 against the FP64 oracle: two tubes and two boxes (the two smallest
    # of each kind and instances 3 and 35).  Measured: tubes about 1e-6,
    # boxes up to 8.7e-4 (the vortex's steepening fronts); guard 2e-3.
    bw = sorted((i for i, p in enumerate(probs) if p.ny == 1), key=lambda i: probs[i].nx)[:2]
    ot = sorted((i for i, p in enumerate(probs) if p.ny > 1), key=lambda i: probs[i].nx * probs[i].ny)[:2]
    for i in sorted(set(bw + ot + [3, 35])):
        ora = oracle_lib.State(probs[i], form=oracle_lib.LOWSTORE)
        ora.run(100)
        got = b[i].read_fields().cpu().numpy()
        errs = [oracle_lib.rel_l2(got[k], ora.stacked()[k]) for k in range(6)]
        print(f"[batch] instance {i} ({probs[i].nx}x{probs[i].ny}) FP32 vs FP64 oracle rel-L2: "
              + " ".join(f"{e:.2e}" for e in errs), flush=True)
        assert max(errs) <= 2e-3, (i, max(errs))


def test_batch_advance_in_parts_equals_one_call():
    """7 + 8 steps in two launches equal 15 steps of the single runs: a
    launch closes its instances' last step, the next one begins from it."""
    _torch()
    from paper_1710_06423_amd import Batch, Solver, FP32
    probs = _mixed(2, 2, seed=3)
    b = Batch(probs, precision=FP32)
    b.advance(7)
    b.advance(8)
    for i, p in enumerate(probs):
        s = Solver.from_problem(p, precision=FP32)
        s.advance(15)
        assert np.array_equal(b[i].read_fields().cpu().numpy(), s.read_fields().cpu().numpy()), i
        assert b[i].diagnostics()["steps"] == 15
        s.close()
    b.close()


def test_batch_wait_bound_is_reported(monkeypatch):
    """A dependency wait that exceeds its bound abandons the launch and the
    host reports it.  The bound is forced to zero polls from the host, so
    the first wait that is not already satisfied gives up; every block then
    leaves the work queue and the kernel ends normally."""
    _torch()
    from paper_1710_06423_amd import Batch, FP32, sacx
    monkeypatch.setenv("SACX_BATCH_SPIN_LIMIT", "0")
    probs = _mixed(3, 3, seed=4)
    b = Batch(probs, precision=FP32)
    with pytest.raises(sacx.SacxError) as e:
        b.advance(20)
    assert e.value.code == sacx.EDEVICE and "bound" in str(e.value)
    b.close()
