"""GPU parity at the benchmark's full sizes and launch configuration, on
sampled outputs the oracle computes one by one.

A stage of the scheme couples an element only to its four face neighbours
(and the limiter to its neighbours' means), so k stages of an element depend
on the elements within distance k (2k with the limiter). The oracle is run
on a patch around each sampled element: periodic meshes wrap the patch
indices; transmissive meshes clip them at the domain edge, where the patch's
own transmissive boundary coincides with the domain's. The sampled element's
oracle result is then exact, and it is compared element by element with the
GPU's full-mesh result."""

import numpy as np
import pytest

import inputs
from oracle import adjoint, cpr, limiter
from tests.gpu_util import dev, host, make_solver, say, torch

pytestmark = pytest.mark.gpu


def _patch(q, g, I, J, r):
    """Patch of radius r (elements) around (I, J): (patch, its Grid, (I, J)
    position of the centre inside the patch)."""
    if g.bc == "periodic":
        Is = [(I + d) % g.nx for d in range(-r, r + 1)]
        Js = [(J + d) % g.ny for d in range(-r, r + 1)]
        ci, cj = r, r
    else:
        Is = list(range(max(0, I - r), min(g.nx, I + r + 1)))
        Js = list(range(max(0, J - r), min(g.ny, J + r + 1)))
        ci, cj = I - Is[0], J - Js[0]
    sub = q[:, Js][:, :, Is]
    # Patches of periodic meshes wrap their indices, so the centre's
    # dependencies never reach the patch boundary; clipped patches of
    # transmissive meshes share the domain's boundary. Either way a
    # transmissive patch grid gives the centre its full-mesh value.
    pg = cpr.Grid(P=g.P, nx=len(Is), ny=len(Js), x0=0.0, x1=g.dx * len(Is), y0=0.0,
                  y1=g.dy * len(Js), bc="transmissive", gamma=g.gamma)
    return np.ascontiguousarray(sub), pg, ci, cj


def _fp32_scale(q, g):
    """(2/h)(||D||_inf + 2||g'||_inf) max|F|: the size of the terms the
    residual is formed from (and whose rounding it carries)."""
    from oracle import euler, tables
    T = tables.get(g.P)
    normD = np.max(np.sum(np.abs(T.D), axis=1))
    normg = max(np.max(np.abs(T.gLp)), np.max(np.abs(T.gRp)))
    Fmax = max(np.max(np.abs(euler.flux_x(q, g.gamma))), np.max(np.abs(euler.flux_y(q, g.gamma))))
    return 2.0 / min(g.dx, g.dy) * (normD + 2 * normg) * Fmax


def _samples(g, n, seed):
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (g.nx - 1, g.ny - 1), (g.nx // 2, g.ny // 2), (7, 8), (8, 7)}
    while len(pts) < n:
        pts.add((int(rng.integers(g.nx)), int(rng.integers(g.ny))))
    return sorted(pts)


def _vortex(g):
    x, y = g.coords()
    return inputs.Vortex().conserved(x, y)


@pytest.mark.parametrize("P,n,prec", [(3, 256, "fp64"), (3, 256, "fp32_bulk"),
                                      (4, 1024, "fp64"), (4, 1024, "fp32_bulk")])
def test_fullsize_residual_sampled(P, n, prec):
    g = cpr.Grid(P=P, nx=n, ny=n)
    say("fullsize residual", P, n, prec)
    q = _vortex(g)
    s = make_solver(g, precision=prec)
    R = host(s.residual(dev(q))).astype(np.float64)
    del s
    # the residual cancels terms of size scale = (2/h)(|D| + 2|g'|) max|F|;
    # both sides round them in different orders
    scale = _fp32_scale(q, g)
    bound64 = 16 * 2.0 ** -53 * scale
    bound32 = 64 * 2.0 ** -24 * scale
    for I, J in _samples(g, 24, seed=P * 100 + n):
        sub, pg, ci, cj = _patch(q, g, I, J, 1)
        Ro = cpr.residual(sub, pg)[:, cj, ci]
        Rg = R[:, J, I]
        if prec == "fp64":
            assert np.max(np.abs(Rg - Ro)) <= bound64, (I, J)
        else:
            # float32 forward-error scale of the residual (see test_gpu_residual)
            assert np.max(np.abs(Rg - Ro)) <= bound32, (I, J)


@pytest.mark.parametrize("P,n,dt", [(3, 256, 5.8e-4), (4, 1024, 1e-4)])
def test_fullsize_rk3_step_sampled(P, n, dt):
    """One SSP-RK3 step of the full mesh (three fused stage kernels, the
    benchmark's launch configuration); each sampled element is checked
    against the oracle's step on a 7x7 patch."""
    g = cpr.Grid(P=P, nx=n, ny=n)
    say("fullsize rk3 step", P, n)
    q = _vortex(g)
    s = make_solver(g)
    qd = dev(q)
    s.step(qd, dt)
    qg = host(qd)
    I0 = s.integrals(dev(q))
    I1 = s.integrals(qd)
    del s, qd
    assert np.max(np.abs(I1 - I0) / np.abs(I0)) < 1e-13
    for I, J in _samples(g, 12, seed=7 + P):
        sub, pg, ci, cj = _patch(q, g, I, J, 3)
        qo = cpr.rk3_step(sub, dt, pg)[:, cj, ci]
        assert np.max(np.abs(qg[:, J, I] - qo)) <= 1e-12 * np.max(np.abs(qo)), (I, J)


def test_fullsize_riemann_limited_run():
    """P=2 four-quadrant Riemann problem, 512x512 transmissive, TVB M=10,
    CFL 0.1 with the device dt, to t=0.3. Checks: the device time reaches
    t_end exactly, the state stays physical and finite, the solution keeps
    the problem's diagonal symmetry exactly, and the first limited step matches the
    oracle on sampled 13x13 patches (flags away from their thresholds)."""
    n = 512
    g = cpr.Grid(P=2, nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc="transmissive")
    x, y = g.coords()
    q0 = inputs.riemann_quadrants(x, y)
    say("fullsize riemann 512 limited")
    s = make_solver(g, limiter=True, tvb_m=10.0, cfl=0.1, t_end=0.3)
    s.set_time(0.0)
    qd = dev(q0)
    s.limit(qd)
    q_lim0 = host(qd)
    np.testing.assert_allclose(q_lim0, limiter.limit(q0, g, M=10.0), rtol=0, atol=1e-13)
    s.step(qd, 0.0, limit=True)
    t1, dt1 = s.get_time()
    q1 = host(qd)
    for I, J in _samples(g, 10, seed=3):
        sub, pg, ci, cj = _patch(q_lim0, g, I, J, 6)
        lim_p = lambda z, pg=pg: limiter.limit(z, pg, M=10.0)
        qo = cpr.rk3_step(sub, dt1, pg, limit=lim_p)[:, cj, ci]
        assert np.max(np.abs(q1[:, J, I] - qo)) <= 1e-11 * np.max(np.abs(qo)), (I, J)
    steps = 1
    t = t1
    while t < 0.3 * (1 - 1e-14) and steps < 20000:
        for _ in range(200):          # past t_end the steps leave q unchanged
            s.step(qd, 0.0, limit=True)
        steps += 200
        t, _ = s.get_time()
    assert abs(t - 0.3) < 1e-14
    qT = host(qd)
    assert np.all(np.isfinite(qT))
    rho = qT[0]
    from oracle import euler
    assert rho.min() > 0 and euler.pressure(qT, 1.4).min() > 0
    # every kernel rounds transposed data identically, so the diagonal
    # symmetry of the data survives 4600 limited steps bit for bit
    qt = qT[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3)
    assert np.array_equal(qt, qT)
    print(f"riemann 512: {steps} steps to t=0.3, rho in [{rho.min():.4f}, {rho.max():.4f}]")


def test_fullsize_adjoint_gradient():
    """P=3 128x128 vortex with seeded density noise (sigma 1e-3, seed 0):
    the gradient of J = 1/2 ||rho(T) - rho_exact(T)||^2_w through 400 steps
    of dt=1e-3 (checkpoint every 50) agrees with central differences of the
    GPU forward on 16 random directions, and on a 5-step horizon with the
    oracle's stored-state adjoint element by element."""
    from paper_1709_01619_amd import Rollout
    t = torch()
    g = cpr.Grid(P=3, nx=128, ny=128)
    x, y = g.coords()
    V = inputs.Vortex()
    q0 = V.conserved(x, y)
    q0[0] += inputs.gaussian_perturbation(q0[0].shape, 1e-3, 0)
    say("fullsize adjoint 128 P3")
    s = make_solver(g)
    W = s.quad_weights()

    def misfit(qT, rho_ex):
        return 0.5 * float(((qT[0] - rho_ex) ** 2 * W).sum().item())

    # short horizon against the oracle
    n5, dt = 5, 1e-3
    rho5 = dev(V.conserved(x, y, n5 * dt)[0])
    qd = dev(q0).requires_grad_(True)
    qT = Rollout.apply(qd, s, dt, n5, 2)
    J = 0.5 * ((qT[0] - rho5) ** 2 * W).sum()
    J.backward()
    J_o, g_o = adjoint.gradient(q0, dt, n5, g, host(rho5))
    assert abs(J.item() - J_o) <= 1e-11 * J_o
    assert np.max(np.abs(host(qd.grad) - g_o)) <= 1e-10 * np.max(np.abs(g_o))

    # full horizon: finite differences of the GPU forward
    N = 400
    rhoN = dev(V.conserved(x, y, N * dt)[0])
    qd = dev(q0).requires_grad_(True)
    qT = Rollout.apply(qd, s, dt, N, 50)
    J = 0.5 * ((qT[0] - rhoN) ** 2 * W).sum()
    J.backward()
    grad = qd.grad.detach()

    def fwd(q):
        z = q.clone()
        for _ in range(N):
            s.step(z, dt)
        return misfit(z, rhoN)

    q0d = dev(q0)
    worst = 0.0
    for d in inputs.random_directions(g.shape, range(1000, 1016)):
        dd = dev(d)
        h = 1e-6 * float(q0d.abs().max()) / float(dd.abs().max())
        fd = (fwd(q0d + h * dd) - fwd(q0d - h * dd)) / (2 * h)
        ad = float((grad * dd).sum().item())
        worst = max(worst, abs(fd - ad) / abs(ad))
    print(f"adjoint FD worst relative error over 16 directions: {worst:.2e}")
    assert worst <= 1e-6


def test_max_size_periodic_tiling():
    """Largest size class: P=4 on 4700x4700 periodic elements, 2.2e9
    unknowns (17.7 GB per state), so flat indices pass 2^31 and the last tile
    column is ragged (4700 = 587 x 8 + 4). The state is a seeded random
    47x47-element block repeated 100 x 100 times; the periodic scheme is
    translation invariant, so the residual and one RK3 step of the large mesh
    must equal the oracle's on the block, repeated, at every element, and the
    conservation sums must be 10^4 times the block's."""
    t = torch()
    P, nb, rep = 4, 47, 100
    h = 0.01
    gb = cpr.Grid(P=P, nx=nb, ny=nb, x0=0.0, x1=nb * h, y0=0.0, y1=nb * h)
    g = cpr.Grid(P=P, nx=nb * rep, ny=nb * rep, x0=0.0, x1=nb * rep * h, y0=0.0,
                 y1=nb * rep * h)
    qb = inputs.random_state((nb, nb, P + 1, P + 1), seed=4747)
    say("max size: P=4 4700x4700 periodic tiling")
    s = make_solver(g)
    q = dev(qb).repeat(1, rep, rep, 1, 1)
    assert q.numel() == 4 * 4700 * 4700 * 25 and q.is_contiguous()

    def max_tiled_diff(big, small):
        d = 0.0
        sm = dev(small)
        for k in range(4):
            v = big[k].view(rep, nb, rep, nb, P + 1, P + 1)
            d = max(d, float((v - sm[k][None, :, None]).abs().max().item()))
        return d

    Rb = cpr.residual(qb, gb)
    R = s.residual(q)
    scale = _fp32_scale(qb, gb)
    assert max_tiled_diff(R, Rb) <= 16 * 2.0 ** -53 * scale
    del R
    Ib = cpr.integrals(qb, gb)
    I = s.integrals(q)
    assert np.max(np.abs(I - rep * rep * Ib) / np.abs(rep * rep * Ib)) <= 1e-12
    dt = 2e-4
    qb1 = cpr.rk3_step(qb, dt, gb)
    s.step(q, dt)
    assert max_tiled_diff(q, qb1) <= 1e-12 * np.max(np.abs(qb1))
    del q, s


def test_c4_adjoint_gradient_fd_16_directions():
    """The adjoint workload at its full size: P=3 vortex on 128x128 with a
    seeded Gaussian perturbation (sigma 1e-3, seed 0) of the initial
    density, 400 steps of dt=1e-3, checkpoint every 50; the FP64 gradient of
    the density misfit at t=0.4 through Rollout against central differences
    of the same misfit along 16 seeded random directions, each from two
    forward runs of the same kernels (replayed from one 400-step graph).
    Relative agreement 1e-6: the step h = 1e-6 max|q0| / max|d| leaves a
    truncation error O(h^2) and a rounding error of the misfit difference
    far below that."""
    from paper_1709_01619_amd import Rollout, Solver
    t = torch()
    say("c4 adjoint fd 16 directions")
    s = Solver(3, 128, 128)
    x, y = s.coords()
    V = inputs.Vortex()
    xn, yn = x.cpu().numpy(), y.cpu().numpy()
    q0n = V.conserved(xn, yn)
    q0n[0] += inputs.gaussian_perturbation(q0n[0].shape, 1e-3, 0)
    rho_ex = t.from_numpy(V.conserved(xn, yn, 0.4)[0]).cuda()
    W = s.quad_weights()
    q0 = t.from_numpy(q0n).cuda()
    qa = q0.clone().requires_grad_(True)
    qT = Rollout.apply(qa, s, 1e-3, 400, 50)
    (0.5 * ((qT[0] - rho_ex) ** 2 * W).sum()).backward()
    grad = qa.grad.detach()
    buf = q0.clone()
    run = s.capture_steps(buf, 1e-3, 400)

    def misfit(start):
        buf.copy_(start)
        run.replay()
        return float((0.5 * ((buf[0] - rho_ex) ** 2 * W).sum()).item())

    worst = 0.0
    for d in inputs.random_directions(q0n.shape, range(2000, 2016)):
        dd = t.from_numpy(d).cuda()
        h = 1e-6 * float(q0.abs().max()) / float(dd.abs().max())
        fd = (misfit(q0 + h * dd) - misfit(q0 - h * dd)) / (2 * h)
        ad = float((grad * dd).sum())
        worst = max(worst, abs(fd - ad) / abs(ad))
    print(f"c4 adjoint: 16 directions, max relative FD - adjoint difference {worst:.2e}")
    assert worst <= 1e-6
