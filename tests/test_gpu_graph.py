"""Steps captured into a HIP graph (StepGraph) and replayed: every replay,
with eager work and synchronisation in between, leaves the state bit for bit
where the eager calls leave it."""

import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("case", ["ot_fp64", "ot_fp32", "brio_wu", "stratified"])
def test_solver_graph_replays_match_eager(case):
    torch = _torch()
    from paper_1710_06423_amd import FP32, FP64, Solver
    prec = FP32 if case == "ot_fp32" else FP64
    prob = {"ot_fp64": lambda: W.orszag_tang(96, ny=80), "ot_fp32": lambda: W.orszag_tang(96, ny=80),
            "brio_wu": lambda: W.brio_wu(500),
            "stratified": lambda: W.stratified_atmosphere(64, 72, amp=0.05, b_b=(0.1, 0.4))}[case]()
    print(f"case: graph {case}", flush=True)
    side = torch.cuda.Stream()
    g_solver = Solver.from_problem(prob, precision=prec, stream=side)
    eager = Solver.from_problem(prob, precision=prec)
    graph = g_solver.graph(5)
    for k in range(1, 4):
        graph.replay()
        eager.advance(5)
        torch.cuda.synchronize()
        a, b = g_solver.read_fields(), eager.read_fields()
        da, db = g_solver.diagnostics(), eager.diagnostics()
        assert torch.equal(a, b), k
        assert da["steps"] == db["steps"] == 5 * k and da["t"] == db["t"]
    # eager calls on the captured context continue from the replayed state
    g_solver.advance(3)
    eager.advance(3)
    assert torch.equal(g_solver.read_fields(), eager.read_fields())


def test_decomposed_graph_replays_match_undivided():
    torch = _torch()
    from paper_1710_06423_amd import DecomposedSolver, Solver
    prob = W.orszag_tang(100, ny=72)
    side = torch.cuda.Stream()
    dec = DecomposedSolver(prob, [0, 45, 100], [0, 36, 72], stream=side)
    one = Solver.from_problem(prob)
    graph = dec.graph(2)
    for k in range(1, 4):
        graph.replay()
        one.advance(2)
        torch.cuda.synchronize()
        assert torch.equal(dec.read_fields(), one.read_fields()), k
        d = dec.diagnostics()[1][0]
        assert d["steps"] == 2 * k and d["t"] == one.diagnostics()["t"]
    dec.advance(1)
    one.advance(1)
    assert torch.equal(dec.read_fields(), one.read_fields())


def test_graph_needs_its_own_stream_and_no_profiling():
    torch = _torch()
    from paper_1710_06423_amd import Solver
    s = Solver.from_problem(W.orszag_tang(32), stream=torch.cuda.default_stream())
    with pytest.raises(ValueError):
        s.graph(1)
    t = Solver.from_problem(W.orszag_tang(32), stream=torch.cuda.Stream())
    t.profile_enable(True)
    with pytest.raises(ValueError):
        t.graph(1)
    t.profile_enable(False)
    t.graph(1).replay()
    torch.cuda.synchronize()
    assert t.diagnostics()["steps"] == 1


def test_tensors_shared_across_streams_are_ordered():
    """A context on its own stream reads inputs that kernels on the caller's
    stream have just produced, and hands back outputs the caller's stream
    reads at once: the binding orders the two streams both ways."""
    torch = _torch()
    from paper_1710_06423_amd import Solver
    prob = W.orszag_tang(512, ny=384)
    ref = Solver.from_problem(prob)
    ref.advance(3)
    side = Solver.from_problem(prob, stream=torch.cuda.Stream(), init=False)
    host = torch.stack([torch.from_numpy(prob.fields[k]) for k in W.FIELDS])
    for rep in range(3):
        # produced by a chain of kernels on the caller's (default) stream,
        # each exact (scaling by powers of two), so f equals the host arrays
        f = host.cuda() * 2.0
        for _ in range(20):
            f = f * 1.0
        f = f * 0.5
        side.init_state(f)
        side.advance(3, sync=False)
        out = side.read_fields()
        assert torch.equal(out * 1.0, ref.read_fields()), rep


def test_closing_a_context_with_queued_work_keeps_fresh_allocations_intact():
    """A context on its own stream is closed, and its workspace dropped,
    while steps are still queued: closing waits for them, and the freed
    block goes back to the context stream's pool, so a tensor allocated and
    filled right afterwards on the caller's stream keeps its values."""
    torch = _torch()
    from paper_1710_06423_amd import Solver
    prob = W.orszag_tang(512, ny=512)
    for rep in range(3):
        s = Solver.from_problem(prob, stream=torch.cuda.Stream())
        nbytes = s.workspace.numel()
        s.advance(20, sync=False)
        s.close()
        del s
        x = torch.full((nbytes,), 7, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        assert int((x != 7).sum()) == 0, rep
