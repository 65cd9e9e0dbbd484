"""Decomposed stepping (paper section 3, Fig. 1): a domain split into
subdomain contexts that exchange their halo strips before every stage and
share one time step evolves bit for bit as the undivided domain, which
itself follows the FP64 oracle bit for bit.

All subdomains run on one GPU, on one stream; the exchange buffers are what
several GPUs would send each other.
"""

import dataclasses

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


def _whole(prob, nsteps, **kw):
    from paper_1710_06423_amd import Solver
    s = Solver.from_problem(prob, **kw)
    s.advance(nsteps)
    f = s.read_fields()
    d = s.diagnostics()
    s.close()
    return f, d


def _decomposed(prob, xcuts, ycuts, nsteps, device_max=True, native=True, **kw):
    from paper_1710_06423_amd import DecomposedSolver
    dec = DecomposedSolver(prob, xcuts, ycuts, **kw)
    dec.advance(nsteps, device_max=device_max, native=native)
    f = dec.read_fields()
    d = dec.diagnostics()
    dec.close()
    return f, d


def _check(torch, prob, xcuts, ycuts, nsteps, label, device_max=True, native=True, **kw):
    print(f"case: {label} cuts x {xcuts} y {ycuts} steps {nsteps} device_max={device_max} native={native} {kw}",
          flush=True)
    ref, dref = _whole(prob, nsteps, **kw)
    got, dgot = _decomposed(prob, xcuts, ycuts, nsteps, device_max=device_max, native=native, **kw)
    nd = int((got != ref).sum())
    print(f"[decomposed] {label}: {nd} elements differ", flush=True)
    assert nd == 0, label
    for row in dgot:
        for d in row:
            assert d["steps"] == dref["steps"] and d["t"] == dref["t"] and d["dt"] == dref["dt"]
    return got


@pytest.mark.parametrize("xcuts,ycuts", [
    ([0, 50, 128], [0, 40, 96]),          # 2 x 2 as in the paper's figure, uneven
    ([0, 128], [0, 31, 64, 96]),          # strips along y, x periodic locally
    ([0, 3, 70, 128], [0, 96]),           # strips along x, one of 3 columns (the halo depth)
    ([0, 40, 80, 128], [0, 30, 66, 96]),  # 3 x 3
    ([0, 128], [0, 96]),                  # one subdomain: no exchange side at all
])
@pytest.mark.parametrize("native", [True, False])
def test_periodic_orszag_tang(xcuts, ycuts, native):
    """Through the library's domain object (native) and through the
    stage-level calls driven from Python."""
    torch = _torch()
    _check(torch, W.orszag_tang(128, ny=96), xcuts, ycuts, 12, "OT periodic", native=native)


@pytest.mark.parametrize("device_max", [True, False])
def test_periodic_matches_oracle(oracle_lib, device_max):
    """The decomposed run against the oracle directly, with the maxima over
    the subdomains reduced on the device or on the host."""
    torch = _torch()
    prob = W.orszag_tang(96, ny=80)
    got = _check(torch, prob, [0, 33, 96], [0, 47, 80], 15, "OT vs oracle", device_max=device_max).cpu().numpy()
    ora = oracle_lib.State(prob, form=oracle_lib.LOWSTORE)
    ora.run(15)
    assert np.array_equal(got, ora.stacked())


@pytest.mark.parametrize("bc", [(OPEN, OPEN, 0, 0), (0, 0, OPEN, OPEN), (OPEN,) * 4])
def test_open_boundaries(bc):
    """Open outer sides with exchange sides inside (the corners of a y strip
    come from an x exchange next to an open fill), and the same domain as a
    single subdomain."""
    torch = _torch()
    prob = W.random_smooth(90, 70, seed=5, bc=bc)
    _check(torch, prob, [0, 41, 90], [0, 33, 70], 10, f"random smooth bc {bc}")
    _check(torch, prob, [0, 90], [0, 70], 10, f"random smooth bc {bc}, one subdomain")


@pytest.mark.parametrize("native", [True, False])
def test_brio_wu_pieces(native):
    """A 1-D shock tube cut into three pieces (open ends)."""
    torch = _torch()
    _check(torch, W.brio_wu(800), [0, 250, 551, 800], [0, 1], 40, "Brio-Wu", native=native)


def test_domain_object_rejects_bad_layouts():
    """sacx_domain_* argument checks: sides and strips that do not match, a
    short or misaligned buffer, a step in progress."""
    torch = _torch()
    import ctypes
    from paper_1710_06423_amd import EXCHANGE, OPEN, Solver, sacx
    lib = sacx.load_library()
    prob = W.orszag_tang(64, ny=40)

    def sub(nx, ny, bc):
        g = sacx.make_grid(nx, ny, 0.0, 1.0, 0.0, 1.0)
        s = Solver(g, sacx.make_params(5 / 3), bc)
        f = torch.stack([torch.from_numpy(prob.fields[k][:ny, :nx].copy()) for k in W.FIELDS]).cuda()
        s.init_state(f)
        return s

    def size(subs, px, py):
        arr = (ctypes.c_void_p * len(subs))(*[s.ctx.value for s in subs])
        n = ctypes.c_size_t(0)
        return lib.sacx_domain_buffer_size(px, py, arr, ctypes.byref(n)), n.value, arr

    x2 = (EXCHANGE, EXCHANGE, 0, 0)
    a, b = sub(32, 40, x2), sub(32, 40, x2)
    rc, need, arr = size([a, b], 2, 1)
    assert rc == sacx.OK and need > 0
    buf = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr() + (-buf.data_ptr()) % 256
    d = ctypes.c_void_p(None)
    assert lib.sacx_domain_create(2, 1, arr, ctypes.c_void_p(base), need - 8, ctypes.byref(d)) == sacx.ENOSPC
    assert lib.sacx_domain_create(2, 1, arr, ctypes.c_void_p(base + 8), need, ctypes.byref(d)) == sacx.EINVAL
    assert lib.sacx_domain_create(2, 1, arr, ctypes.c_void_p(base), need, ctypes.byref(d)) == sacx.OK
    a.stage(None)                                 # a step begun by hand ...
    assert lib.sacx_domain_advance(d, 1) == sacx.ESTATE
    for _ in range(3):
        a.fill_boundaries(0)
        a.fill_boundaries(1)
        a.stage(None)                             # ... and finished
    assert lib.sacx_domain_advance(d, 1) == sacx.OK
    b.set_boundaries((EXCHANGE, EXCHANGE, OPEN, OPEN))   # no longer the layout the domain checked
    assert lib.sacx_domain_advance(d, 1) == sacx.ESTATE
    b.set_boundaries(x2)
    assert lib.sacx_domain_advance(d, 1) == sacx.OK
    assert lib.sacx_domain_destroy(d) == sacx.OK
    # an interior side that is not EXCHANGE; strips of different lengths; the same context twice
    c = sub(32, 40, (OPEN, OPEN, 0, 0))
    assert size([a, c], 2, 1)[0] == sacx.EINVAL
    e = sub(32, 24, x2)
    assert size([a, e], 2, 1)[0] == sacx.EINVAL
    assert size([a, a], 2, 1)[0] == sacx.EINVAL
    assert lib.sacx_domain_advance(None, 1) == sacx.EINVAL
    assert lib.sacx_domain_destroy(None) == sacx.OK


@pytest.mark.parametrize("variant", ["no_hd", "no_cross", "gravity", "one_thread_tile"])
def test_scheme_variants(variant):
    torch = _torch()
    prob = W.orszag_tang(100, ny=72)
    kw = {}
    if variant == "no_hd":
        kw = dict(hd_on=False)
    elif variant == "no_cross":
        kw = dict(hd_cross_on=False)
    elif variant == "gravity":
        prob = W.with_gravity(prob, (0.3, -0.8))
    if variant != "one_thread_tile":
        _check(torch, prob, [0, 45, 100], [0, 36, 72], 10, variant, **kw)
        return
    # the one-thread tile in every subdomain and in the undivided run
    from paper_1710_06423_amd import DecomposedSolver, Solver
    s = Solver.from_problem(prob)
    s.set_column_split(False)
    s.advance(10)
    ref = s.read_fields()
    dec = DecomposedSolver(prob, [0, 45, 100], [0, 36, 72])
    for row in dec.subs:
        for sub in row:
            sub.set_column_split(False)
    dec.advance(10)
    assert torch.equal(dec.read_fields(), ref)


def test_fp32_decomposed_equals_undivided():
    """FP32 bulk: the decomposed run equals the undivided FP32 run bit for
    bit (the FP64 time step is the same, every cell sees the same inputs)."""
    torch = _torch()
    from paper_1710_06423_amd import FP32
    _check(torch, W.orszag_tang(128, ny=80), [0, 64, 128], [0, 37, 80], 12, "OT FP32", precision=FP32)


def test_stage_calls_reject_misuse():
    """Argument and order checks of the stage-level calls."""
    torch = _torch()
    from paper_1710_06423_amd import EXCHANGE, Solver, SacxError, Batch
    from paper_1710_06423_amd import sacx
    prob = W.orszag_tang(32)
    s = Solver.from_problem(prob)

    def code(fn, *a):
        with pytest.raises(SacxError) as e:
            fn(*a)
        return e.value.code

    assert code(s.fill_boundaries, 2) == sacx.EINVAL
    assert code(s.set_boundaries, (3, 0, 0, 0)) == sacx.EINVAL
    assert code(s.set_boundaries, (0, EXCHANGE, 0, 0)) == sacx.EINVAL   # periodic sides come in pairs
    assert code(s.stage, (float("nan"), 1.0)) == sacx.EINVAL
    assert code(s.stage, (0.0, 1.0)) == sacx.EINVAL
    s.set_boundaries((EXCHANGE,) * 4)
    assert code(s.advance, 1) == sacx.ESTATE
    s.set_boundaries((0,) * 4)
    assert s.stage(None) == 1                 # a step begun stage by stage ...
    assert code(s.advance, 1) == sacx.ESTATE  # ... must be finished that way
    s.fill_boundaries(0)
    s.fill_boundaries(1)
    assert s.stage(None) == 2
    for st in (3, 4):
        s.fill_boundaries(0)
        s.fill_boundaries(1)
        assert s.stage((123.0, 456.0)) == st   # c_max is only read at stage 1
    s.advance(1)
    assert s.diagnostics()["steps"] == 2
    lib = s.lib
    c = torch.zeros(2, dtype=torch.float64, device=s.device)
    assert lib.sacx_stage(s.ctx, None, 1, None) == sacx.EINVAL          # a device c_max must be given
    assert lib.sacx_stage(s.ctx, c.data_ptr() + 4, 1, None) == sacx.EINVAL   # misaligned
    assert lib.sacx_stage(s.ctx, c.data_ptr(), 2, None) == sacx.EINVAL
    # the device max equals the host read-back
    s.wave_speeds_max(c)
    assert tuple(c.cpu().tolist()) == s.wave_speeds()
    # a bad device value stops this subdomain's stepping, reported as non-physical
    c.fill_(float("nan"))
    for _ in range(4):
        s.fill_boundaries(0)
        s.fill_boundaries(1)
        s.stage(c)
    d = s.diagnostics()
    assert d["nonphys"] and d["steps"] == 2
    s.close()
    # a background cannot have exchange sides; a small direction neither
    bg = Solver.from_problem(W.stratified_atmosphere(16, 20))
    assert code(bg.set_boundaries, (0, 0, EXCHANGE, EXCHANGE)) == sacx.EUNSUP
    bg.close()
    thin = Solver.from_problem(W.orszag_tang(2, ny=16))
    assert code(thin.set_boundaries, (EXCHANGE, EXCHANGE, 0, 0)) == sacx.EUNSUP
    thin.close()
    with pytest.raises(SacxError) as e:
        Batch([dataclasses.replace(W.orszag_tang(32), bc=(EXCHANGE,) * 4)])
    assert e.value.code == sacx.EUNSUP


def test_stage_by_stage_equals_advance():
    """A single context stepped stage by stage with its own boundary fills
    and its own wave speeds equals sacx_advance."""
    torch = _torch()
    from paper_1710_06423_amd import Solver
    prob = W.random_smooth(60, 44, seed=9, bc=(OPEN, OPEN, 0, 0))
    a = Solver.from_problem(prob)
    a.advance(8)
    b = Solver.from_problem(prob)
    for _ in range(8):
        for _st in range(4):
            b.fill_boundaries(0)
            b.fill_boundaries(1)
            b.stage(None)
    assert torch.equal(a.read_fields(), b.read_fields())
    assert a.diagnostics()["t"] == b.diagnostics()["t"]
