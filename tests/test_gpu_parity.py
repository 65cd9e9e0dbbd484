"""GPU parity: the HIP path against the FP64 CPU oracle, through the C ABI.

FP64 bar: relative L2 per field <= 1e-12 after the whole run, at sizes that
span several 250-column tiles and row strips with a ragged tail.  Because the
hyper-diffusion coefficient amplifies rounding differences, the FP64 device
path reproduces the IEEE operation sequence of the oracle's low-storage form
(the four-array RK4 arrangement with reciprocals), and these tests require
bit-for-bit equality with it (exact=True).  The CPU pins tie that form to the
oracle's paper form (textbook RK4 combine, divisions as written); the
`test_paper_form_*` cases below compare the device with the paper form
directly, where rounding is not amplified: many steps without
hyper-diffusion, a few with it.
"""

import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_run(prob, nsteps, t_end=0.0, **kw):
    _torch()
    from paper_1710_06423_amd import Solver
    s = Solver.from_problem(prob, **kw)
    done, t = s.advance(nsteps, t_end)
    out = s.read_fields().cpu().numpy()
    return s, out, done, t


def oracle_run(oracle, prob, nsteps, t_end=0.0, **kw):
    s = oracle.State(prob, form=oracle.LOWSTORE, **kw)
    s.run(nsteps, t_end)
    return s


def assert_parity(oracle, gpu_fields, ora_state, tol=TOL64, label="", exact=True):
    ref = ora_state.stacked()
    errs = [oracle.rel_l2(gpu_fields[k], ref[k]) for k in range(6)]
    ndiff = int(np.sum(gpu_fields != ref))
    print(f"[parity] {label} rel-L2 per field: " + " ".join(f"{e:.2e}" for e in errs)
          + f"; elements differing: {ndiff} of {ref.size}", flush=True)
    for k, e in enumerate(errs):
        assert e <= tol, (label, W.FIELDS[k], e)
    if exact:
        assert ndiff == 0, (label, ndiff)
    return errs


def test_library_loads_on_gpu():
    torch = _torch()
    from paper_1710_06423_amd import load_library
    lib = load_library()
    assert lib.sacx_abi_version() == 3
    assert torch.cuda.get_device_properties(0).gcnArchName.startswith("gfx950")


@pytest.mark.parametrize("hd_on,nsteps", [(False, 100), (True, 3)])
def test_paper_form_orszag_tang(oracle_lib, hd_on, nsteps):
    """OT 256 x 192 against the oracle's paper form: 100 steps without
    hyper-diffusion, 3 with it, relative L2 per field <= 1e-12."""
    print(f"case: paper form OT 256x192 hd={hd_on} steps={nsteps}", flush=True)
    prob = W.orszag_tang(256, ny=192)
    s, out, done, t = gpu_run(prob, nsteps, hd_on=hd_on)
    ora = oracle_lib.State(prob, hd_on=hd_on, form=oracle_lib.PAPER)
    ora.run(nsteps)
    assert done == nsteps and abs(t - ora.t) <= 1e-13 * ora.t
    assert_parity(oracle_lib, out, ora, label=f"paper form OT256x192 hd={hd_on}", exact=False)


def test_paper_form_brio_wu(oracle_lib):
    """Brio-Wu 800 with hyper-diffusion, 3 steps, against the paper form."""
    print("case: paper form brio_wu 800 3 steps", flush=True)
    prob = W.brio_wu(800)
    s, out, done, t = gpu_run(prob, 3)
    ora = oracle_lib.State(prob, form=oracle_lib.PAPER)
    ora.run(3)
    assert_parity(oracle_lib, out, ora, label="paper form BW-800 3 steps", exact=False)


def test_brio_wu_800_parity(oracle_lib):
    """Brio-Wu 800 cells, gamma = 2, open ends, CFL 0.3, HD on, to t = 0.1."""
    print("case: brio_wu 800 t_end=0.1", flush=True)
    prob = W.brio_wu(800)
    s, out, done, t = gpu_run(prob, 100000, t_end=0.1)
    ora = oracle_run(oracle_lib, prob, 100000, t_end=0.1)
    assert done == ora.steps and t == ora.t
    assert_parity(oracle_lib, out, ora, label="BW-800")
    assert np.all(out[4] == 0.75)


@pytest.mark.parametrize("hd_on,cross,bg", [(True, True, False), (False, True, False), (True, False, False),
                                           (True, True, True)])
def test_orszag_tang_ragged_parity(oracle_lib, hd_on, cross, bg):
    """OT on a 300 x 136 grid (two column tiles, ragged last tile and strip), 40 steps."""
    print(f"case: OT 300x136 hd={hd_on} cross={cross} bg={bg}", flush=True)
    prob = W.orszag_tang(300, ny=136)
    if bg:
        gamma = prob.gamma
        rho0, p0 = 25 / (36 * math.pi), 5 / (12 * math.pi)
        bb = (0.05, -0.08)
        prob = W.split_background(prob, rho0 / 2, p0 / (2 * (gamma - 1)) + 0.5 * (bb[0] ** 2 + bb[1] ** 2), bb)
    s, out, done, t = gpu_run(prob, 40, hd_on=hd_on, hd_cross_on=cross)
    ora = oracle_run(oracle_lib, prob, 40, hd_on=hd_on, hd_cross_on=cross)
    assert done == 40 and t == ora.t
    assert_parity(oracle_lib, out, ora, label=f"OT300x136 hd={hd_on} cross={cross} bg={bg}")


def test_open_boundaries_2d_parity(oracle_lib):
    print("case: random smooth 257x70 open", flush=True)
    prob = W.random_smooth(257, 70, seed=4, bc=(W.problems.OPEN,) * 4)
    s, out, done, t = gpu_run(prob, 30)
    ora = oracle_run(oracle_lib, prob, 30)
    assert_parity(oracle_lib, out, ora, label="open 257x70")


def test_mixed_boundaries_parity(oracle_lib):
    print("case: random smooth 64x251 open x periodic y", flush=True)
    prob = W.random_smooth(64, 251, seed=9, bc=(W.problems.OPEN, W.problems.OPEN, 0, 0))
    s, out, done, t = gpu_run(prob, 30)
    ora = oracle_run(oracle_lib, prob, 30)
    assert_parity(oracle_lib, out, ora, label="open-x 64x251")


def test_brio_wu_along_y_parity(oracle_lib):
    print("case: brio_wu along y 1x400", flush=True)
    prob = W.brio_wu(400, along_y=True)
    s, out, done, t = gpu_run(prob, 100000, t_end=0.05)
    ora = oracle_run(oracle_lib, prob, 100000, t_end=0.05)
    assert done == ora.steps
    assert_parity(oracle_lib, out, ora, label="BW-y 400")


def test_uniform_state_bit_exact():
    print("case: uniform 300x40", flush=True)
    prob = W.uniform_state(300, 40)
    s, out, done, t = gpu_run(prob, 20)
    for k, name in enumerate(W.FIELDS):
        assert np.array_equal(out[k], prob.fields[name]), name


def test_determinism_and_resume():
    torch = _torch()
    from paper_1710_06423_amd import Solver
    print("case: OT 256 determinism/resume", flush=True)
    prob = W.orszag_tang(256)
    a = Solver.from_problem(prob)
    a.advance(20)
    fa = a.read_fields()
    b = Solver.from_problem(prob)
    b.advance(20)
    assert torch.equal(fa, b.read_fields())
    c = Solver.from_problem(prob)
    c.advance(8)
    mid = c.read_fields()
    t_mid = c.diagnostics()["t"]
    d = Solver.from_problem(prob, init=False)
    d.init_state(mid, t0=t_mid)
    d.advance(12)
    assert torch.equal(fa, d.read_fields())
    assert d.diagnostics()["t"] == a.diagnostics()["t"]


def test_conservation_sums(oracle_lib):
    _torch()
    from paper_1710_06423_amd import Solver
    print("case: OT 320x200 conservation", flush=True)
    prob = W.orszag_tang(320, ny=200)
    s = Solver.from_problem(prob)
    d0 = s.diagnostics()
    s.advance(50)
    d1 = s.diagnostics()
    cfg = oracle_lib.make_cfg(prob, form=oracle_lib.LOWSTORE)
    ref0 = oracle_lib.sums(cfg, [prob.fields[k] for k in W.FIELDS])
    absum = oracle_lib.sums(cfg, [np.abs(prob.fields[k]) for k in W.FIELDS])
    assert np.allclose(d0["sums"], ref0, rtol=1e-13, atol=1e-13 * absum.max())
    assert np.all(np.abs(np.array(d1["sums"]) - np.array(d0["sums"])) <= 1e-12 * np.maximum(absum, 1e-300))
    assert d1["steps"] == 50 and d1["nonphys"] == 0


def test_nonphysical_state_reported():
    _torch()
    from paper_1710_06423_amd import Solver, sacx
    print("case: nonphysical", flush=True)
    prob = W.orszag_tang(64)
    prob.fields["e"][5, 7] = 0.0
    s = Solver.from_problem(prob)
    rc, done, t = s.advance_rc(5)
    assert rc == sacx.ENONPHYS and done == 0
    assert s.diagnostics()["nonphys"] == 1
    assert np.array_equal(s.read_fields().cpu().numpy()[3], prob.fields["e"])


def test_wave_speeds_match_oracle(oracle_lib):
    _torch()
    from paper_1710_06423_amd import Solver
    prob = W.orszag_tang(200, ny=120)
    s = Solver.from_problem(prob)
    d = s.diagnostics()
    cx, cy, cmax, dt = oracle_lib.State(prob, form=oracle_lib.LOWSTORE).wavespeed()
    assert d["c_x"] == cx and d["c_y"] == cy
    s.advance(1)
    assert s.diagnostics()["dt"] == dt


def test_halo_pack_unpack_bit_exact():
    torch = _torch()
    from paper_1710_06423_amd import Solver
    print("case: halo pack/unpack", flush=True)
    prob = W.random_smooth(37, 29, seed=1)
    s = Solver.from_problem(prob)
    f = prob.stacked()
    G = 3
    for side in range(4):
        buf = s.halo_buffer(side)
        s.halo_pack(side, buf)
        b = buf.cpu().numpy()
        if side < 2:
            b = b.reshape(6, G, prob.ny)
            c0 = 0 if side == 0 else prob.nx - G
            ref = np.stack([f[:, :, c0 + g] for g in range(G)], axis=1)
            assert np.array_equal(b, ref)
        else:
            b = b.reshape(6, G, prob.nx + 2 * G)
            r0 = 0 if side == 2 else prob.ny - G
            cols = np.arange(-G, prob.nx + G) % prob.nx      # x halo of a periodic state
            ref = np.stack([f[:, r0 + g, :][:, cols] for g in range(G)], axis=1)
            assert np.array_equal(b, ref)
    # unpack a known pattern into the x+ ghosts and read it back through a pack of ... the interior is unchanged
    buf = s.halo_buffer(1)
    buf.copy_(torch.arange(buf.numel(), dtype=buf.dtype, device=buf.device))
    s.halo_unpack(1, buf)
    assert np.array_equal(s.read_fields().cpu().numpy(), f)


def test_fp32_path_error_budget(oracle_lib):
    """FP32 bulk arithmetic (FP64 dt and sums): per-field relative L2 <= 1e-5
    against the FP64 oracle on OT (30 steps on 256^2; longer and full-size
    cases below)."""
    _torch()
    from paper_1710_06423_amd import Solver, FP32
    print("case: OT 256 fp32", flush=True)
    prob = W.orszag_tang(256)
    s = Solver.from_problem(prob, precision=FP32)
    s.advance(30)
    out = s.read_fields().cpu().numpy()
    ora = oracle_run(oracle_lib, prob, 30)
    assert_parity(oracle_lib, out, ora, tol=1e-5, label="OT-256 FP32 30 steps", exact=False)


def test_fp32_512_100_steps_error_growth(oracle_lib):
    """FP32 bulk against the FP64 oracle over 100 steps of OT 512^2 (t = 0.16,
    fifteen times the simulated time of the 8000^2 benchmark run).  The
    ratio coefficient amplifies the FP32 rounding as the run goes on; the
    per-field relative L2 measured here is 5e-6 to 1.3e-5, guarded at 1.6e-5.
    The 1e-5 budget is the benchmark run's (t = 0.01 at 8000^2; the slow
    8000^2 test), not this longer one's."""
    _torch()
    from paper_1710_06423_amd import Solver, FP32
    print("case: OT 512 fp32 100 steps", flush=True)
    prob = W.orszag_tang(512)
    s = Solver.from_problem(prob, precision=FP32)
    s.advance(100)
    out = s.read_fields().cpu().numpy()
    ora = oracle_run(oracle_lib, prob, 100)
    assert_parity(oracle_lib, out, ora, tol=1.6e-5, label="OT-512 FP32 100 steps", exact=False)


@pytest.mark.slow
def test_fp32_8000_error_budget():
    """The 8000^2 workload in FP32 bulk against the FP64 path (bit-identical to
    the oracle, see the sampled parity test) after 100 steps: per-field
    relative L2 <= 1e-5."""
    torch = _torch()
    from paper_1710_06423_amd import Solver, FP32, FP64
    print("case: OT 8000 fp32 vs fp64 100 steps", flush=True)
    prob = W.orszag_tang(8000)
    a = Solver.from_problem(prob, precision=FP32)
    b = Solver.from_problem(prob, precision=FP64)
    del prob
    a.advance(100)
    b.advance(100)
    x, y = a.read_fields(torch.float64), b.read_fields(torch.float64)
    for k in range(6):
        rel = float(torch.linalg.vector_norm(x[k] - y[k]) / torch.linalg.vector_norm(y[k]))
        print(f"[parity] OT-8000 FP32 field {k}: rel-L2 {rel:.3e}", flush=True)
        assert rel <= 1e-5


@pytest.mark.slow
def test_orszag_tang_1024_200_steps_parity(oracle_lib):
    """The 1024^2, 200-step Orszag-Tang workload against the oracle."""
    print("case: OT 1024 200 steps", flush=True)
    prob = W.orszag_tang(1024)
    s, out, done, t = gpu_run(prob, 200)
    ora = oracle_run(oracle_lib, prob, 200)
    assert done == 200
    assert_parity(oracle_lib, out, ora, label="OT-1024x200")


@pytest.mark.slow
def test_orszag_tang_8000_sampled_parity(oracle_lib):
    """The 8000^2 FP64 workload in the launch configuration the benchmark
    times: after 99 GPU steps, the oracle recomputes step 100 on sampled
    patches (tile seams, strip seams, domain corners across the periodic
    wrap, interior) from the GPU state, with the dt and c_max it reduces from
    the whole 8000^2 state itself; the GPU's step 100 must match bit for bit."""
    torch = _torch()
    from paper_1710_06423_amd import Solver
    n = 8000
    print("case: OT 8000 sampled step 99 -> 100", flush=True)
    prob = W.orszag_tang(n)
    s = Solver.from_problem(prob)
    cfg = oracle_lib.make_cfg(prob, form=oracle_lib.LOWSTORE)
    del prob
    done, t = s.advance(99)
    assert done == 99
    u99 = s.read_fields().cpu().numpy()
    d99 = s.diagnostics()
    cx, cy, cmax, dt = oracle_lib.wavespeed(cfg, list(u99))
    assert (cx, cy) == (d99["c_x"], d99["c_y"])
    s.advance(1)
    assert s.diagnostics()["dt"] == dt
    u100 = s.read_fields().cpu().numpy()
    rng = np.random.default_rng(100)
    w = 40
    centres = [(0, 0), (n - 20, n - 20), (249, 3000), (250, 127), (4000, 4000), (7999, 5000), (3000, 7999)]
    centres += [tuple(int(v) for v in rng.integers(0, n, size=2)) for _ in range(9)]
    for (ci, cj) in centres:
        ii = np.arange(ci - w // 2 - 12, ci + w // 2 + 12) % n
        jj = np.arange(cj - w // 2 - 12, cj + w // 2 + 12) % n
        patch = [u99[k][np.ix_(jj, ii)] for k in range(6)]
        ref = oracle_lib.step_patch(cfg, patch, None, dt, cmax)
        got = np.stack([u100[k][np.ix_(jj[12:-12], ii[12:-12])] for k in range(6)])
        nd = int(np.sum(got != ref))
        print(f"[parity] 8000^2 patch at ({ci},{cj}): elements differing {nd} of {ref.size}", flush=True)
        assert nd == 0
    # whole-field sanity of the final state
    assert np.all(np.isfinite(u100))


@pytest.mark.parametrize("nt,ty", [(64, 7), (128, 7), (128, 40), (256, 16)])
def test_background_multiwave_parity(oracle_lib, nt, ty):
    """Background-on contexts with one- to four-wave blocks and short strips
    (many strip starts) follow the oracle bit for bit, HD and cross terms on:
    an earlier build gave wrong values in the first rows of each strip with
    multi-wave blocks, which this case would show."""
    _torch()
    from paper_1710_06423_amd import Solver
    print(f"case: background OT 200x96 launch ({nt}, {ty})", flush=True)
    prob = W.split_background(W.orszag_tang(200, ny=96), 0.1, 0.1, (0.05, -0.02))
    s = Solver.from_problem(prob)
    s.set_launch(nt, ty)
    s.advance(15)
    ora = oracle_run(oracle_lib, prob, 15)
    assert_parity(oracle_lib, s.read_fields().cpu().numpy(), ora, label=f"background launch ({nt}, {ty})")


@pytest.mark.parametrize("shape", [(64, 16), (128, 8), (256, 37), (256, 256)])
def test_launch_shape_does_not_change_results(oracle_lib, shape):
    """Any block width / strip height gives the same bits as the oracle."""
    _torch()
    from paper_1710_06423_amd import Solver
    prob = W.orszag_tang(300, ny=136)
    s = Solver.from_problem(prob)
    s.set_launch(*shape)
    s.advance(12)
    ora = oracle_run(oracle_lib, prob, 12)
    assert_parity(oracle_lib, s.read_fields().cpu().numpy(), ora, label=f"launch {shape}")


@pytest.mark.parametrize("shape", [(64, 7), (128, 256), (256, 33), (128, 1), (64, 2), (256, 3), (128, 4)])
@pytest.mark.parametrize("cross,background", [(True, False), (False, False), (True, True)])
def test_column_split_matches_one_thread_tiles(shape, cross, background):
    """The two-threads-per-column tile (x and y roles) and the one-thread tile
    give the same bits over every stage of several steps (time step included),
    for block widths and strip heights that leave ragged tiles and strips
    (down to strips of one to four rows, shorter than the warm-up), on mixed
    open and periodic boundaries; with a background and gravity too."""
    torch = _torch()
    from paper_1710_06423_amd import Solver
    print(f"case: split vs one-thread {shape} cross={cross} background={background}", flush=True)
    if background:
        prob = W.stratified_atmosphere(301, 138, amp=0.08, b_b=(0.2, 0.5))
    else:
        prob = W.random_smooth(301, 138, seed=11, bc=(W.problems.OPEN, W.problems.OPEN, 0, 0))
    res = []
    for split in (True, False):
        s = Solver.from_problem(prob, hd_cross_on=cross)
        s.set_launch(*shape)
        s.set_column_split(split)
        s.advance(9)
        d = s.diagnostics()
        res.append((s.read_fields(), d["t"], d["dt"]))
        s.close()
    assert torch.equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1] and res[0][2] == res[1][2]


@pytest.mark.parametrize("shape,kind", [((2, 2), "periodic"), ((2, 5), "periodic"), ((5, 2), "periodic"),
                                        ((3, 3), "periodic"), ((4, 7), "periodic"), ((7, 4), "periodic"),
                                        ((6, 5), "open"), ((130, 3), "open")])
def test_tiny_grids_parity(oracle_lib, shape, kind):
    """Grids smaller than the stencil or a tile (one block, most threads in
    the apron, strips shorter than the warm-up, periodic images wrapping more
    than once) follow the oracle bit for bit with both FP64 tiles."""
    _torch()
    from paper_1710_06423_amd import Solver
    print(f"case: tiny {shape} {kind}", flush=True)
    bc = (0,) * 4 if kind == "periodic" else (W.problems.OPEN,) * 4
    prob = W.random_smooth(*shape, seed=3, bc=bc)
    ora = oracle_run(oracle_lib, prob, 12)
    for split in (True, False):
        s = Solver.from_problem(prob)
        s.set_column_split(split)
        s.advance(12)
        assert_parity(oracle_lib, s.read_fields().cpu().numpy(), ora, label=f"tiny {shape} {kind} split={split}")
        s.close()
