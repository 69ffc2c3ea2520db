"""GPU parity of the paper's nodal DG (Section 2.4), the "gll_lp" scheme:
Gauss-Lobatto points, the derivative of the flux interpolant and the Radau
lift (the exact-mass-matrix lift of NDG), against the oracle. Tolerances as
for the Gauss-Legendre scheme (same formulas, other nodes): 1e-12 relative
for the residual, steps and transposes. The paper's NDG errors (Tables 2
and 3) are checked with the other schemes in test_gpu_chain.py."""

import numpy as np
import pytest

import inputs
from oracle import adjoint, cpr, euler, limiter, tables
from tests.gpu_util import dev, host, make_solver, rel_err, say, torch
from tests.test_gpu_limiter_adjoint import _blurred_riemann, _margins

pytestmark = pytest.mark.gpu

NDG = cpr.GLL_LP
MESHES = [(1, 1), (2, 2), (3, 5), (8, 8), (9, 8), (13, 11), (17, 3), (1, 17), (23, 1), (33, 2)]


def _transpose(a):
    return np.ascontiguousarray(a[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3))


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("mesh", MESHES, ids=lambda m: f"{m[0]}x{m[1]}")
def test_ndg_residual_fp64_matches_oracle(mesh, P, bc):
    nx, ny = mesh
    g = cpr.Grid(P=P, nx=nx, ny=ny, x0=0.0, x1=2.0, y0=-1.0, y1=0.5, bc=bc, scheme=NDG)
    q = inputs.random_state((ny, nx, P + 1, P + 1), seed=3000 + 10 * P + nx)
    say("ndg residual fp64", P, nx, ny, bc)
    R = cpr.residual(q, g)
    Rg = host(make_solver(g).residual(dev(q)))
    assert rel_err(Rg, R) <= 1e-12


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_ndg_residual_fp32_bulk_error_bound(P):
    g = cpr.Grid(P=P, nx=13, ny=9, x0=0.0, x1=2.0, y0=0.0, y1=1.0, scheme=NDG)
    q = inputs.random_state((9, 13, P + 1, P + 1), seed=3500 + P)
    say("ndg residual fp32_bulk", P)
    R = cpr.residual(q, g)
    Rg = host(make_solver(g, precision="fp32_bulk").residual(dev(q))).astype(np.float64)
    T = tables.get(P, "gll")
    normD = np.max(np.sum(np.abs(T.D), axis=1))
    normg = max(np.max(np.abs(T.gLp)), np.max(np.abs(T.gRp)))
    Fmax = max(np.max(np.abs(euler.flux_x(q, 1.4))), np.max(np.abs(euler.flux_y(q, 1.4))))
    scale = 2.0 / min(g.dx, g.dy) * (normD + 2 * normg) * Fmax
    assert np.max(np.abs(Rg - R)) <= 64 * 2.0 ** -24 * scale


@pytest.mark.parametrize("P,prec", [(1, "fp64"), (2, "fp64"), (3, "fp64"), (4, "fp64"),
                                    (3, "fp32_bulk")])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_ndg_residual_transpose_bitwise_and_conservative(P, prec, bc):
    g = cpr.Grid(P=P, nx=21, ny=21, x0=0.0, x1=2.0, y0=0.0, y1=2.0, bc=bc, scheme=NDG)
    q = inputs.random_state((21, 21, P + 1, P + 1), seed=3600 + P)
    say("ndg transpose bitwise", P, prec, bc)
    s = make_solver(g, precision=prec)
    r = host(s.residual(dev(q)))
    rt = host(s.residual(dev(_transpose(q))))
    assert np.array_equal(rt, _transpose(r))
    if bc == "periodic" and prec == "fp64":
        tot = s.integrals(dev(r))
        assert np.max(np.abs(tot)) < 1e-13 * np.max(np.abs(r)) * 6.0


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_ndg_rk3_step_matches_oracle(P, bc):
    g = cpr.Grid(P=P, nx=11, ny=10, x0=0.0, x1=10.0, y0=0.0, y1=10.0, bc=bc, scheme=NDG)
    x, y = g.coords()
    q = inputs.Vortex().conserved(x, y)
    say("ndg rk3 step", P, bc)
    s = make_solver(g)
    qd = dev(q)
    q1 = q
    for _ in range(3):
        q1 = cpr.rk3_step(q1, 0.01, g)
        s.step(qd, 0.01)
    assert rel_err(host(qd), q1) <= 1e-12


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("mesh", [(1, 1), (3, 5), (9, 8), (13, 11)], ids=lambda m: f"{m[0]}x{m[1]}")
def test_ndg_residual_vjp_matches_oracle(mesh, P, bc):
    nx, ny = mesh
    g = cpr.Grid(P=P, nx=nx, ny=ny, x0=0.0, x1=2.0, y0=0.0, y1=1.5, bc=bc, scheme=NDG)
    q = inputs.random_state((ny, nx, P + 1, P + 1), seed=3700 + P + nx)
    v = np.random.default_rng(3800 + P).standard_normal(g.shape)
    say("ndg vjp", P, nx, ny, bc)
    ref = adjoint.residual_vjp(q, v, g)
    out = host(make_solver(g).residual_vjp(dev(q), dev(v)))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("P", [2, 3])
def test_ndg_adjoint_step_matches_oracle(P):
    g = cpr.Grid(P=P, nx=10, ny=9, scheme=NDG)
    x, y = g.coords()
    q = inputs.Vortex().conserved(x, y)
    lam = np.random.default_rng(3900 + P).standard_normal(g.shape)
    say("ndg adjoint step", P)
    ref = adjoint.rk3_adjoint_step(q, 0.01, lam, g)
    out = host(make_solver(g).adjoint_step(dev(q), 0.01, dev(lam)))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_ndg_limiter_matches_oracle(P):
    g = cpr.Grid(P=P, nx=21, ny=19, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc="transmissive",
                 scheme=NDG)
    q = _blurred_riemann(g)
    say("ndg limiter", P)
    ql, flags = limiter.limit(q, g, M=10.0, return_flags=True)
    s = make_solver(g, limiter=True, tvb_m=10.0)
    qd = dev(q)
    fd = torch().zeros((g.ny, g.nx), dtype=torch().int32, device="cuda")
    n = s.limit(qd, flags=fd, count=True)
    fg = host(fd).astype(bool)
    safe = _margins(q, g, 10.0) > 1e-9
    assert flags.any()
    assert np.array_equal(fg[safe], flags[safe])
    assert n == int(fg.sum())
    both = safe & (fg == flags)
    assert np.max(np.abs(host(qd)[:, both] - ql[:, both])) <= 1e-13 * max(1.0, np.max(np.abs(ql)))
