"""HIP-graph capture of the step path (Solver.capture_steps): each replay
of a recorded run equals the same run launched kernel by kernel, bit for
bit (the same kernels on the same data), with eager work and
synchronisations between the replays; recording itself runs nothing."""

import numpy as np
import pytest

import inputs
from oracle import cpr
from tests.gpu_util import dev, host, make_solver, say, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P,prec", [(1, "fp64"), (2, "fp64"), (3, "fp64"), (3, "fp32_bulk"),
                                    (4, "fp64")])
def test_captured_steps_equal_eager(P, prec):
    t = torch()
    g = cpr.Grid(P=P, nx=20, ny=20)
    x, y = g.coords()
    q0 = inputs.Vortex().conserved(x, y)
    say("graph steps", P, prec)
    s = make_solver(g, precision=prec)
    qg = dev(q0)
    graph = s.capture_steps(qg, 1e-3, 10)
    t.cuda.synchronize()
    assert np.array_equal(host(qg), q0)
    start = dev(q0)
    for _ in range(3):
        qe = start.clone()
        for _ in range(10):
            s.step(qe, 1e-3)
        t.cuda.synchronize()
        qg.copy_(start)
        graph.replay()
        t.cuda.synchronize()
        assert t.equal(qg, qe)
        start = qe + 0.0   # the next replay starts from a new state


def test_captured_limited_device_dt_steps_equal_eager():
    """The C3 step (limiter after every stage, CFL dt formed on the device)
    on the four-quadrant Riemann problem: replays from the same state and
    time reach the same state, time and troubled count as eager steps."""
    t = torch()
    g = cpr.Grid(P=2, nx=32, ny=32, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc="transmissive")
    x, y = g.coords()
    q0 = inputs.riemann_quadrants(x, y)
    say("graph limited device-dt steps")
    s = make_solver(g, limiter=True, tvb_m=10.0, cfl=0.1, t_end=0.3)
    qs = dev(q0)
    s.limit(qs)
    qg = qs.clone()
    graph = s.capture_steps(qg, 0.0, 8, limit=True)
    for _ in range(3):
        s.set_time(0.0)
        s.troubled_total(reset=True)
        qe = qs.clone()
        for _ in range(8):
            s.step(qe, 0.0, limit=True)
        te, dte = s.get_time()
        ne = s.troubled_total(reset=True)
        s.set_time(0.0)
        qg.copy_(qs)
        graph.replay()
        tg, dtg = s.get_time()
        ng = s.troubled_total(reset=True)
        assert t.equal(qg, qe)
        assert (tg, dtg, ng) == (te, dte, ne)
        assert te > 0.0 and ne > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32_bulk"])
def test_headline_size_graph_replay_equals_eager(prec):
    """At the timed workload's full size (P=3 vortex on 256x256, the
    benchmark's dt) the benchmark's graph replay gives the same state, bit
    for bit, as the same steps launched kernel by kernel; the full-size
    parity tests check the kernel-by-kernel state against the oracle."""
    t = torch()
    g = cpr.Grid(P=3, nx=256, ny=256)
    x, y = g.coords()
    q0 = dev(inputs.Vortex().conserved(x, y))
    say("headline graph replay", prec)
    s = make_solver(g, precision=prec)
    qe = q0.clone()
    for _ in range(12):
        s.step(qe, 5.8e-4)
    qg = q0.clone()
    graph = s.capture_steps(qg, 5.8e-4, 12)
    graph.replay()
    t.cuda.synchronize()
    assert t.equal(qg, qe)


def test_capture_rejects_what_a_step_rejects():
    """Recording runs the step's own argument checks: a limited step on a
    context without a limiter, or a device dt without a CFL number, raises
    the library's error while recording; the state is left untouched."""
    from paper_1709_01619_amd import _lib
    g = cpr.Grid(P=2, nx=8, ny=8)
    x, y = g.coords()
    q0 = inputs.Vortex().conserved(x, y)
    say("graph capture errors")
    s = make_solver(g)
    q = dev(q0)
    with pytest.raises(_lib.CprError) as ei:
        s.capture_steps(q, 1e-3, 2, limit=True)
    assert ei.value.status == _lib.CPR_EUNSUPPORTED
    with pytest.raises(_lib.CprError) as ei:
        s.capture_steps(q, 0.0, 2)
    assert ei.value.status == _lib.CPR_EINVAL
    with pytest.raises(ValueError):
        s.capture_steps(q, 1e-3, 0)
    assert np.array_equal(host(q), q0)
    s.step(q, 1e-3)   # the context still works after the aborted recordings
    torch().cuda.synchronize()


def test_graph_keeps_its_solver_and_state_alive():
    """A recorded graph's kernels use the solver's scratch and the state
    through raw pointers: the StepGraph holds both, so dropping every other
    reference frees neither; close() refuses while the graph exists, and the
    replay equals eager steps on a fresh solver."""
    import gc
    import weakref

    t = torch()
    g = cpr.Grid(P=2, nx=16, ny=12)
    x, y = g.coords()
    q0 = inputs.Vortex().conserved(x, y)
    say("graph lifetime")
    s = make_solver(g)
    qg = dev(q0)
    graph = s.capture_steps(qg, 1e-3, 4)
    with pytest.raises(RuntimeError):
        s.close()
    ws, wq = weakref.ref(s), weakref.ref(qg)
    del s, qg
    gc.collect()
    assert ws() is not None and wq() is not None
    graph.replay()
    t.cuda.synchronize()
    ref = make_solver(g)
    qe = dev(q0)
    for _ in range(4):
        ref.step(qe, 1e-3)
    t.cuda.synchronize()
    assert t.equal(graph.q, qe)
    del graph
    gc.collect()
    assert ws() is None
